#!/usr/bin/env python3
"""Benchmark of the subgraph-isomorphism hot path on one MI355X.

One step = one pass of the query path over the workload: every query of the
query set, one at a time (filter, plan, join levels, result rows in HBM
with their digest), on a data graph resident in HBM.  The device structures
(PCSR for every edge label, signature table) are built from the edge list
in HBM before the timed region -- preprocessing, which the paper keeps out
of query time -- and their build time is reported as build_ms.

Workload (default "ba1m"): Barabasi-Albert graph with 1,000,000 vertices and
9,999,945 undirected edges, 32 vertex labels Zipf(1.1), 8 edge labels
uniform; 100 random-walk queries with 6..12 vertices.  Synthetic, seeded.

Prints ONE JSON line.  Fields beyond the common contract:
  roofline      the kernel with the largest share of device time in the timed
                steps: algorithmic bytes / its summed HIP-event duration,
                against the 8 TB/s HBM peak
  cpu_baseline  the CPU oracle (count + digest of every embedding) on the
                same graph and queries, all host threads
  queries_per_s, latency_ms {p50, p99}: per query, submit -> result ready
  parity        GPU counts and digests against the stored oracle values
  batched       1,024 mixed queries on the same graph, one at a time vs one
                batch (fused persistent tiers + level-synchronous engine)
  ablations     the paper's join ablations and this design's switches on the
                single-query workload
  serving       the request loop on an R-MAT scale-22 graph: saturation
                throughput, then Poisson arrivals at 0.5 / 0.8 / 1.2 times it,
                with p50 / p99 latency (arrival -> answer ready on device)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "embeddings/s and queries/s (batched vs single) on one MI355X; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# kernels of the path's own steps: signature filter, PCSR locate, join
# (set subtraction + intersections), link (Prealloc-Combine table write), and
# the fused workgroup that runs locate/join/link for small tables
HOT_KERNELS = ("k_filter", "k_locate", "k_join", "k_link", "k_fused_levels")

# sources each kernel is compiled from: the stored HBM counter readings of a
# kernel (profiles/traffic.json) are used only while these files are unchanged
CSRC = os.path.join(ROOT, "paper_1906_03420_amd", "csrc")
KERNEL_SOURCES = {
    "k_fused_levels": ("fused.hip", "fused.h", "join_device.h", "gsi_internal.h"),
    "k_fused_chunks": ("fused.hip", "fused.h", "join_device.h", "gsi_internal.h"),
    "k_filter": ("query.hip", "gsi_internal.h"),
    "k_locate": ("query.hip", "join_device.h", "gsi_internal.h"),
    "k_join": ("query.hip", "join_device.h", "scan_device.h", "gsi_internal.h"),
    "k_link": ("query.hip", "join_device.h", "gsi_internal.h"),
}


def sources_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, ()):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, scaled by the copy
    probe) from the committed counter runs, or None when the kernel's
    sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if kernel not in KERNEL_SOURCES or not os.path.exists(path):
        return None
    rec = json.load(open(path)).get("kernels", {}).get(kernel)
    if not rec or rec.get("sources_sha256") != sources_digest(kernel):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


WORKLOAD_TEXT = {
    "ba1m": "BA graph 1,000,000 vertices / 9,999,945 edges, 32 vertex labels Zipf(1.1), 8 edge labels uniform; "
            "100 random-walk queries of 6-12 vertices; single-query path",
    "er1k": "ER graph 1,000 vertices / 5,000 edges, 4 vertex labels, 2 edge labels; 8 random-walk queries of 4 "
            "vertices; single-query path",
    "rmat23": "R-MAT scale 23, 8,388,608 vertices / 100,000,000 edges, 100 vertex + 20 edge labels Zipf(1.1); "
              "the 12-vertex walk and dense queries with stored oracle values; single-query path",
}


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    n = os.cpu_count() or 1
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, min(n, 16))


def load_golden(name):
    path = os.path.join(ROOT, "tests", "golden", "%s.json" % name)
    if not os.path.exists(path):
        return None
    return json.load(open(path))


def make_workload(name):
    """The workload's graph and queries; with stored oracle values, exactly
    the queries they cover (index and accepted attempt of each)."""
    import workloads as w
    g = w.config_graph(name)
    mk = w.QueryMaker(g)
    gold = load_golden(name)
    qs = []
    if gold:
        for x in gold["queries"]:
            qs.append(w.config_query(g, name, x["index"], attempt=x["attempt"], maker=mk))
    else:
        for i in range(w.CONFIGS[name]["nq"]):
            qs.append(w.config_query(g, name, i, maker=mk))
    mk.close()
    return g, qs, gold


def cpu_baseline(g, qs, threads, min_s=10.0):
    """The oracle on the same graph and queries: adjacency build once, then
    whole passes over the queries until at least min_s seconds."""
    import oracle
    t0 = time.perf_counter()
    og = oracle.OracleGraph(g)
    tb = time.perf_counter() - t0
    total, passes = 0, 0
    t1 = time.perf_counter()
    while passes == 0 or time.perf_counter() - t1 < min_s:
        for q in qs:
            total += og.match(q, threads=threads, tuples=False).count
        passes += 1
    dt = time.perf_counter() - t1
    og.close()
    return dict(value=total / dt, unit="embeddings/s", cores=threads, kind="oracle",
                sample="%d whole passes over the %d queries (count + digest of every embedding), %.1f s; "
                       "adjacency build %.2f s not counted" % (passes, len(qs), dt, tb))


def batched_section(args, vl_t, s_t, d_t, l_t, g, arena):
    """The 1,024-query mixed workload on the same resident graph, run one
    query at a time and as one batch; both timed over --steps passes after
    --warmup passes (the autotuner runs in the first warm-up pass)."""
    import numpy as np
    import torch
    import workloads as w
    import paper_1906_03420_amd as gsi
    name = "ba1m_batch"
    gold = load_golden(name)
    mk = w.QueryMaker(g)
    qs = [w.config_query(g, name, x["index"], attempt=x["attempt"], maker=mk) for x in gold["queries"]]
    mk.close()
    ctx = gsi.Context(arena)
    dg = ctx.load_device(g.n, vl_t, s_t, d_t, l_t)

    def ok(counts):
        return all(c == x["count"] and [str(d[0]), str(d[1])] == x["digest"] for (c, d), x in zip(counts, gold["queries"]))

    def sequential():
        out = []
        for q in qs:
            r = dg.query(q)
            out.append((r.count, r.digest))
            r.free()
        torch.cuda.synchronize()
        return out

    def batched():
        b = dg.batch(qs)
        out = [(b.count(i), b.digest(i)) for i in range(len(qs))]
        info = b.info()
        b.free()
        torch.cuda.synchronize()
        return out, info

    tune = None
    parity = True
    for i in range(max(1, args.warmup)):
        if i == 0:
            tune = dg.tune(qs, sample=256)
        parity &= ok(sequential())
        parity &= ok(batched()[0])
    t0 = time.perf_counter()
    for _ in range(args.steps):
        parity &= ok(sequential())
    t_seq = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, info = batched()
        parity &= ok(out)
    t_bat = (time.perf_counter() - t0) / args.steps
    dg.free()
    ctx.close()
    emb = sum(x["count"] for x in gold["queries"])
    return dict(workload="BA graph (same as above) with 1,024 random-walk queries of 4-16 vertices, shapes tree / "
                         "walk with a cycle / dense; %d embeddings per pass" % emb,
                sequential=dict(queries_per_s=len(qs) / t_seq, embeddings_per_s=emb / t_seq, ms_per_pass=t_seq * 1e3),
                batched=dict(queries_per_s=len(qs) / t_bat, embeddings_per_s=emb / t_bat, ms_per_pass=t_bat * 1e3),
                speedup=t_seq / t_bat, schedule=info["schedule"], autotune=tune,
                tiers=dict(empty=info["empty"], tier1=info["tier1"], tier2=info["tier2"], per_level=info["per_level"]),
                parity="bit-exact counts+digests vs oracle, both paths, %d/%d" % (len(qs), len(qs)) if parity
                else "MISMATCH")


def ablation_section(args, vl_t, s_t, d_t, l_t, g, qs, gold, arena):
    """The paper's ablations (Tables V-VII) on the same 100 queries, one at a
    time: the per-level kernels as built, then with N(v,l) found by binary
    search in the compressed representation instead of PCSR, with two-step
    output instead of Prealloc-Combine, and without LDS-staged row writes;
    plus this design's own switches (fused small-table workgroup off, the
    first edge of Algorithm 4 for every row).  Each variant must give the
    oracle's counts and digests."""
    import torch
    import paper_1906_03420_amd as gsi
    ctx = gsi.Context(arena)
    dg = ctx.load_device(g.n, vl_t, s_t, d_t, l_t, gsi.GSI_GRAPH_KEEP_CR)
    variants = [("default", 0), ("level_first_edge", gsi.GSI_LEVEL_FIRST_EDGE), ("per_level", gsi.GSI_NO_FUSED),
                ("per_level+cr_lookup", gsi.GSI_NO_FUSED | gsi.GSI_ABL_CR),
                ("per_level+two_step_output", gsi.GSI_NO_FUSED | gsi.GSI_ABL_TWO_STEP),
                ("per_level+unstaged_rows", gsi.GSI_NO_FUSED | gsi.GSI_ABL_NO_STAGING)]

    def run(flags):
        out = []
        t0 = time.perf_counter()
        for q in qs:
            r = dg.query(q, flags=flags)
            out.append((r.count, r.digest))
            r.free()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    res = {}
    ok = True
    for name, flags in variants:
        run(flags)  # warm-up
        best = None
        for _ in range(max(1, args.steps)):
            dt, out = run(flags)
            best = dt if best is None else min(best, dt)
            ok &= all(c == x["count"] and [str(d[0]), str(d[1])] == x["digest"]
                      for (c, d), x in zip(out, gold["queries"]))
        res[name] = dict(ms_per_pass=best * 1e3)
    base = res["per_level"]["ms_per_pass"]
    for name in res:
        res[name]["vs_per_level"] = res[name]["ms_per_pass"] / base
    dg.free()
    ctx.close()
    return dict(workload="the single-query workload above (100 queries, rows written), best of %d passes"
                         % max(1, args.steps), variants=res,
                parity="bit-exact counts+digests vs oracle in every variant" if ok else "MISMATCH")


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def serving_section(args, arena):
    """Continuous batching on the R-MAT scale-22 graph (50M edges, 64 vertex
    and 16 edge labels Zipf(1.1)).  Requests ask queries of the stored pool
    (uniform with repeats).  First every request arrives at once (saturation
    throughput mu); then, for each factor f, requests arrive as a Poisson
    process of rate f*mu.  Latency = answer ready on the device (rows in
    HBM, count and digest on the host) minus arrival.  Every answer is
    checked against the oracle's count and digest for its query."""
    import numpy as np
    import torch
    import workloads as w
    import paper_1906_03420_amd as gsi
    name = "rmat22_serve"
    gold = load_golden(name)
    if not gold or not gold["queries"]:
        return dict(skipped="no stored query pool for %s" % name)
    c = w.CONFIGS[name]
    t = time.perf_counter()
    g = w.config_graph(name)
    mk = w.QueryMaker(g)
    pool = [w.config_query(g, name, x["index"], attempt=x["attempt"], maker=mk) for x in gold["queries"]]
    mk.close()
    want = [(x["count"], x["digest"]) for x in gold["queries"]]
    gen_s = time.perf_counter() - t
    progress("serving graph generated in %.1f s, pool of %d queries" % (gen_s, len(pool)))
    dev = torch.device("cuda:0")
    as_t = lambda a: torch.from_numpy(a.view(np.int32)).to(dev)
    ctx = gsi.Context(arena)
    tensors = [as_t(g.vlabel), as_t(g.src), as_t(g.dst), as_t(g.elabel)]
    dg = ctx.load_device(g.n, *tensors)
    del tensors
    torch.cuda.synchronize()
    n = c["requests"]

    def run(reqs, arrivals):
        srv = dg.server()
        lat = np.zeros(len(reqs))
        by_ticket, paths = {}, {}
        bad = i = done = 0
        t0 = time.perf_counter()
        while done < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and (arrivals is None or arrivals[i] <= now):
                by_ticket[srv.submit(pool[reqs[i]])] = i
                i += 1
            if i == done:  # nothing in the server: wait for the next arrival
                while time.perf_counter() - t0 < arrivals[i]:
                    pass
                continue
            srv.step()
            tnow = time.perf_counter() - t0
            for tk in srv.poll():
                j = by_ticket.pop(tk)
                a = srv.answer(tk)
                lat[j] = tnow - (arrivals[j] if arrivals is not None else 0.0)
                wc, wd = want[reqs[j]]
                bad += a["status"] != 0 or a["count"] != wc or [str(a["digest"][0]), str(a["digest"][1])] != wd
                paths[a["path"]] = paths.get(a["path"], 0) + 1
                srv.release(tk)
                done += 1
        span = time.perf_counter() - t0
        info = srv.info()
        srv.free()
        return span, lat, bad, info, paths

    emb_of = lambda reqs: int(sum(want[r][0] for r in reqs))
    # one query at a time through the single-query path
    reqs0 = w.request_stream(name, 0, n, len(pool))
    for r in reqs0[:32]:
        dg.query(pool[r]).free()
    t = time.perf_counter()
    seq_bad = 0
    for r in reqs0:
        res = dg.query(pool[r])
        seq_bad += (res.count, [str(v) for v in res.digest]) != (want[r][0], want[r][1])
        res.free()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    progress("serving: one at a time %.0f q/s" % (n / t_seq))
    run(reqs0[:256], None)  # warm-up
    span, lat, bad, info, paths = run(reqs0, None)
    mu = n / span
    progress("serving: saturation %.0f q/s" % mu)
    total_bad = bad + seq_bad
    sat = dict(queries_per_s=mu, embeddings_per_s=emb_of(reqs0) / span, p50_ms=float(np.percentile(lat, 50) * 1e3),
               p99_ms=float(np.percentile(lat, 99) * 1e3), steps=info["steps"], level_steps=info["level_steps"],
               paths=paths, admit_ms=info["admit_ms"], level_ms=info["level_ms"], span_ms=span * 1e3)
    rates = []
    for s_i, f in enumerate((0.5, 0.8, 1.2)):
        reqs = w.request_stream(name, s_i + 1, n, len(pool))
        arr = np.cumsum(w.arrival_gaps(name, s_i + 1, n)) / (f * mu)
        span, lat, bad, info, paths = run(reqs, arr)
        total_bad += bad
        rates.append(dict(offered_factor=f, offered_qps=f * mu, achieved_qps=n / span,
                          p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                          max_ms=float(lat.max() * 1e3), steps=info["steps"], level_steps=info["level_steps"],
                          admit_rounds=info["admit_rounds"], peak_predicted_mb=info["peak_predicted"] / 2**20,
                          admit_ms=info["admit_ms"], level_ms=info["level_ms"], span_ms=span * 1e3))
        progress("serving: %.1f x mu -> p50 %.2f ms p99 %.2f ms" % (f, rates[-1]["p50_ms"], rates[-1]["p99_ms"]))
    dg.free()
    ctx.close()
    ks = sorted(set(int(q.k) for q in pool))
    return dict(workload="R-MAT scale 22, %d vertices / %d edges, 64 vertex + 16 edge labels Zipf(1.1); pool of %d "
                         "queries (k %d-%d, tree / walk with a cycle / dense); %d requests per rate"
                         % (g.n, g.m, len(pool), ks[0], ks[-1], n),
                graph_gen_s=gen_s, one_at_a_time=dict(queries_per_s=n / t_seq,
                                                       embeddings_per_s=emb_of(reqs0) / t_seq),
                saturation=sat, speedup_vs_one_at_a_time=mu * t_seq / n, rates=rates,
                parity=("bit-exact counts+digests vs oracle, every request (%d)" % (4 * n + n)) if total_bad == 0
                else "MISMATCH in %d answers" % total_bad)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ba1m", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--queries", type=int, default=0, help="use only the first N queries of the workload (0: all)")
    ap.add_argument("--arena-gb", type=float, default=48.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-sequential comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-ablations", action="store_true", help="skip the ablation runs")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device copy of this size (a reference kernel for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (asked for %d)" % max(args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1906_03420_amd as gsi

    g, qs, gold = make_workload(args.workload)
    if args.queries and args.queries < len(qs):
        qs = qs[:args.queries]
        if gold:
            gold = dict(gold, queries=gold["queries"][:args.queries])
    dev = torch.device("cuda:0")
    as_t = lambda a: torch.from_numpy(a.view(np.int32)).to(dev)
    vl_t, s_t, d_t, l_t = as_t(g.vlabel), as_t(g.src), as_t(g.dst), as_t(g.elabel)
    torch.cuda.synchronize()

    arena = int(args.arena_gb * (1 << 30))
    ctx = None
    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # The data graph is built once (PCSR and signatures, preprocessing that
    # the paper keeps out of query time) and stays resident; its build time
    # is reported beside the metric.  A step is one pass over the queries.
    def build():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dg = ctx.load_device(g.n, vl_t, s_t, d_t, l_t)
        torch.cuda.synchronize()
        return dg, time.perf_counter() - t0

    def step(dg):
        lat, out = [], []
        for q in qs:
            tq = time.perf_counter()
            r = dg.query(q)
            lat.append(time.perf_counter() - tq)
            out.append((r.count, r.digest))
            r.free()
        torch.cuda.synchronize()
        return lat, out

    def matches(out):
        return all(c == q["count"] and [str(d[0]), str(d[1])] == q["digest"] for (c, d), q in zip(out, gold["queries"]))

    # timed region: plain context, no per-launch events
    ctx = gsi.Context(arena)
    build_all = []
    for _ in range(3):
        dg, bt = build()
        build_all.append(bt)
        dg.free()
    dg, bt = build()
    build_all.append(bt)
    parity_ok = None
    for _ in range(args.warmup):
        _, out = step(dg)
        if gold:
            parity_ok = matches(out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat_all, emb = [], 0
    for _ in range(args.steps):
        lat, out = step(dg)
        lat_all += lat
        emb += sum(c for c, _ in out)
        if gold:
            parity_ok = matches(out) if parity_ok is None else (parity_ok and matches(out))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    dg.free()
    ctx.close()

    # roofline: the same steps again with HIP events recorded around every
    # launch on the library's stream
    ctx = gsi.Context(arena, flags=gsi.GSI_CTX_PROFILE)
    dg, _ = build()
    ctx.kernel_stats_reset()  # query kernels only
    tp = time.perf_counter()
    for _ in range(args.steps):
        step(dg)
    prof_ms = (time.perf_counter() - tp) / args.steps * 1e3
    dg.free()
    ks = ctx.kernel_stats()
    ctx.close()
    ks = [k for k in ks if k["launches"]]
    dev_ms = sum(k["total_ms"] for k in ks)
    dom = max((k for k in ks if k["name"] in HOT_KERNELS), key=lambda k: k["total_ms"])
    achieved = dom["alg_bytes"] / (dom["total_ms"] * 1e-3) / 1e9
    large = [k for k in ks if k["name"].endswith("@large") and k["name"].split("@")[0] in HOT_KERNELS]
    large_lines = {k["name"]: dict(launches=k["launches"], ms=round(k["total_ms"], 3),
                                   achieved_gbs=round(k["alg_bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1),
                                   frac=round(k["alg_bytes"] / (k["total_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
                   for k in large}
    lat_ms = np.array(lat_all) * 1e3
    nq_total = len(qs) * args.steps

    res = dict(
        metric=METRIC,
        value=emb / total,
        unit="embeddings/s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=total / args.steps * 1e3,
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="u32",
        data="synthetic",
        config=dict(workload=WORKLOAD_TEXT[args.workload], name=args.workload, queries=len(qs),
                    path="single-query", graph="resident; PCSR and signatures built before timing (build_ms)",
                    embeddings_per_step=emb // args.steps),
        queries_per_s=nq_total / total,
        latency_ms=dict(p50=float(np.percentile(lat_ms, 50)), p99=float(np.percentile(lat_ms, 99)),
                        max=float(lat_ms.max())),
        build_ms=float(np.median(build_all) * 1e3),
        parity=("bit-exact counts+digests vs oracle, %d/%d queries" % (len(qs), len(qs))) if parity_ok
        else ("MISMATCH" if parity_ok is False else "no stored oracle values"),
        roofline=dict(kernel=dom["name"], bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=stored_traffic(dom["name"]),
                      alg_bytes_per_launch=dom["alg_bytes"] / dom["launches"], launches=dom["launches"],
                      avg_launch_us=dom["total_ms"] / dom["launches"] * 1e3,
                      share_of_device_time=dom["total_ms"] / dev_ms if dev_ms else None,
                      limiter=("latency: one 1024-thread workgroup runs every level of a small query"
                               if dom["name"] == "k_fused_levels" else "hbm"),
                      measured="HIP events around every launch in %d profiled steps (%.1f ms/step with events)"
                               % (args.steps, prof_ms),
                      large_launches=large_lines),
        kernels={k["name"]: dict(launches=k["launches"], ms=round(k["total_ms"], 3),
                                 gbs=round(k["alg_bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1) if k["total_ms"] else None)
                 for k in ks},
    )
    progress("single-query path done: %.3g embeddings/s" % res["value"])
    if not args.no_batched:
        res["batched"] = batched_section(args, vl_t, s_t, d_t, l_t, g, arena)
        progress("batched section done")
    if not args.no_ablations and gold:
        res["ablations"] = ablation_section(args, vl_t, s_t, d_t, l_t, g, qs, gold, arena)
        progress("ablations done")
    if not args.no_serving:
        del vl_t, s_t, d_t, l_t
        torch.cuda.empty_cache()
        res["serving"] = serving_section(args, arena)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(g, qs, host_threads())
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

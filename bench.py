#!/usr/bin/env python3
"""Benchmark of the subgraph-isomorphism hot path on one MI355X.

One step = one pass of the query path over the workload: every query of the
query set, one at a time (filter, plan, join levels, result rows in HBM
with their digest), on a data graph resident in HBM.  The device structures
(PCSR for every edge label, signature table) are built from the edge list
in HBM before the timed region -- preprocessing, which the paper keeps out
of query time -- and their build time is reported as build_ms.

Headline workload (default "rmat23"): R-MAT scale 23, 8,388,608 vertices and
100,000,000 undirected edges (a, b, c = 0.57, 0.19, 0.19), 100 vertex and 20
edge labels Zipf(1.1); 50 twelve-vertex random-walk queries (walk and dense
shapes).  Synthetic, seeded.  This is the largest single-GPU configuration
of the metric; the BA-1M single-query workload (1,000,000 vertices,
9,999,945 edges, 100 queries of 6..12 vertices) is a section of its own.

Prints ONE JSON line.  Fields beyond the common contract:
  roofline        the step kernel with the largest summed device time in the
                  timed passes: algorithmic bytes / its summed HIP-event
                  duration, against the 8 TB/s HBM peak; launches of at least
                  16 MiB of algorithmic bytes are also given apart
  cpu_baseline    the CPU oracle (count + digest of every embedding) on a
                  bounded sample of the headline queries, with every host
                  thread this process may use and with one thread; CPU model
  queries_per_s, latency_ms {p50, p99}: per query, submit -> result ready on
                  the device; latency_d2h_ms: the same plus the rows' copy
                  to host memory
  parity          GPU counts and digests against the stored oracle values
  ba1m            the BA-1M single-query workload, same fields
  batched         1,024 mixed queries on the BA-1M graph, one at a time vs
                  one batch (fused persistent tiers + level-synchronous
                  engine), with the engine kernels' roofline
  ablations       the paper's join ablations and this design's switches on
                  the BA-1M single-query workload
  serving         the request loop on an R-MAT scale-22 graph: saturation
                  throughput, then Poisson arrivals at 0.5 / 0.8 / 1.2 times
                  it, with p50 / p99 latency (arrival -> answer ready on
                  device)
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
# (set subtraction + intersections), link (Prealloc-Combine table write), the
# one-pass levels (join, look-back and link in one launch: k_join_pass for an
# inner level, k_join_last for the last), and the fused workgroup that runs
# locate/join/link for small tables
HOT_KERNELS = ("k_filter", "k_locate", "k_join", "k_link", "k_join_pass", "k_join_last", "k_fused_levels")

# sources each kernel is compiled from: the stored HBM counter readings of a
# kernel (profiles/traffic.json) are used only while these files are unchanged
CSRC = os.path.join(ROOT, "paper_1906_03420_amd", "csrc")
KERNEL_SOURCES = {
    "k_fused_levels": ("fused.hip", "fused.h", "join_device.h", "gsi_internal.h"),
    "k_fused_chunks": ("fused.hip", "fused.h", "join_device.h", "gsi_internal.h"),
    "k_filter": ("query.hip", "gsi_internal.h"),
    "k_locate": ("query.hip", "level.h", "join_device.h", "gsi_internal.h"),
    "k_join": ("query.hip", "level.h", "join_device.h", "scan_device.h", "gsi_internal.h"),
    "k_link": ("query.hip", "level.h", "join_device.h", "gsi_internal.h"),
    "k_join_pass": ("query.hip", "level.h", "join_device.h", "scan_device.h", "gsi_internal.h"),
    "k_join_last": ("query.hip", "level.h", "join_device.h", "scan_device.h", "gsi_internal.h"),
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
              "50 twelve-vertex random-walk queries (walk and dense shapes); single-query path",
}


def cpu_share() -> tuple:
    """(threads the oracle may use, nproc): the CPUs this process may run on,
    capped at OMP_NUM_THREADS when it is set (the host's share for one GPU)."""
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    n = min(nproc, int(env)) if env and env.isdigit() else nproc
    return max(1, n), nproc


def cpu_model() -> dict:
    """CPU model, sockets, cores per socket and threads per core (lscpu)."""
    import subprocess
    out = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except Exception:  # lscpu missing: fall back to /proc/cpuinfo
        txt = ""
    keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
            "Thread(s) per core": "threads_per_core", "CPU(s)": "cpus"}
    for line in txt.splitlines():
        k, _, v = line.partition(":")
        if k.strip() in keys:
            out[keys[k.strip()]] = v.strip()
    if "model" not in out and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                out["model"] = line.split(":", 1)[1].strip()
                break
    if "threads_per_core" in out:
        out["smt"] = "on" if out["threads_per_core"] not in ("1", "") else "off"
    return out


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


def pick_sample(gold, budget_s, max_each_s):
    """Indices (into the query list) of a bounded sample for the oracle: the
    queries in index order whose stored oracle time (8 host threads) is at
    most max_each_s, until their sum would pass budget_s."""
    out, tot = [], 0.0
    for i, x in enumerate(gold["queries"]):
        t = float(x.get("oracle_s", 0.0))
        if t > max_each_s or tot + t > budget_s:
            continue
        out.append(i)
        tot += t
    return out


def oracle_leg(og, qs, idx, threads):
    import oracle
    total, t0 = 0, time.perf_counter()
    for i in idx:
        r = og.match(qs[i], threads=threads, tuples=False)
        assert r.status == oracle.OR_OK
        total += r.count
    return total, time.perf_counter() - t0


def cpu_baseline(g, qs, gold, gpu_lat_s):
    """The oracle (count + digest of every embedding) on a bounded sample of
    the headline workload's queries, with all the host threads this process
    may use and with one thread.  gpu_lat_s[i] is the GPU's median latency
    of query i in the timed steps, so the GPU rate on the same sample is
    reported beside it."""
    import oracle
    threads, nproc = cpu_share()
    t0 = time.perf_counter()
    og = oracle.OracleGraph(g)
    tb = time.perf_counter() - t0
    scale = 8.0 / threads  # stored oracle times were taken with 8 threads
    all_idx = pick_sample(gold, 16.0 / scale, 8.0 / scale)
    one_idx = pick_sample(gold, 16.0 / 8.0, 2.0)
    n_all, t_all = oracle_leg(og, qs, all_idx, threads)
    n_one, t_one = oracle_leg(og, qs, one_idx, 1)
    og.close()
    gpu = lambda idx: sum(gold["queries"][i]["count"] for i in idx) / max(1e-12, sum(gpu_lat_s[i] for i in idx))
    return dict(value=n_all / t_all, unit="embeddings/s", cores=threads, kind="oracle",
                sample="%d of the %d queries (those whose oracle time fits a ~15 s budget; indices %s), "
                       "%d embeddings, count + digest of each, %.1f s on %d threads; adjacency build %.1f s "
                       "not counted" % (len(all_idx), len(qs), all_idx, n_all, t_all, threads, tb),
                single_thread=dict(value=n_one / t_one, cores=1, queries=one_idx, embeddings=n_one, seconds=t_one),
                gpu_same_sample=dict(all_threads_sample=gpu(all_idx), single_thread_sample=gpu(one_idx)),
                host=dict(cpu_model(), nproc=nproc, threads_used=threads,
                          note="the oracle uses the CPUs this process may run on, capped at OMP_NUM_THREADS"),
                build="gcc -O3; pthreads, root candidates dealt round-robin to the threads")


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

    def batched(**sched):
        b = dg.batch(qs, **sched)
        counts, digests = b.results()
        out = [(int(c), (int(d[0]), int(d[1]))) for c, d in zip(counts, digests)]
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
    # (answers are checked after each timed loop, not inside it)
    outs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        outs.append(sequential())
    t_seq = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, info = batched()
        outs.append(out)
    t_bat = (time.perf_counter() - t0) / args.steps
    for out in outs:
        parity &= ok(out)
    # the untuned default schedule (256-thread first tier, full occupancy,
    # 4 engine tiles per workgroup) over the same passes
    default = dict(threads=256, grid_scale=8, engine_tiles=4)
    batched(**default)
    outs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out, _ = batched(**default)
        outs.append(out)
    t_def = (time.perf_counter() - t0) / args.steps
    for out in outs:
        parity &= ok(out)
    dg.free()
    ctx.close()
    # one batched pass again with HIP events around every launch
    ctx = gsi.Context(arena, flags=gsi.GSI_CTX_PROFILE)
    dg = ctx.load_device(g.n, vl_t, s_t, d_t, l_t)
    ctx.kernel_stats_reset()
    tp = time.perf_counter()
    batched()
    prof_ms = (time.perf_counter() - tp) * 1e3
    dg.free()
    ks = [k for k in ctx.kernel_stats() if k["launches"]]
    ctx.close()
    emb = sum(x["count"] for x in gold["queries"])
    return dict(workload="BA graph (same as above) with 1,024 random-walk queries of 4-16 vertices, shapes tree / "
                         "walk with a cycle / dense; %d embeddings per pass" % emb,
                sequential=dict(queries_per_s=len(qs) / t_seq, embeddings_per_s=emb / t_seq, ms_per_pass=t_seq * 1e3),
                batched=dict(queries_per_s=len(qs) / t_bat, embeddings_per_s=emb / t_bat, ms_per_pass=t_bat * 1e3),
                speedup=t_seq / t_bat, schedule=info["schedule"], autotune=tune,
                default_schedule=dict(default, ms_per_pass=t_def * 1e3, tuned_vs_default=t_def / t_bat),
                tiers=dict(empty=info["empty"], tier1=info["tier1"], tier2=info["tier2"], per_level=info["per_level"]),
                phases_ms={p: round(info[p], 3) for p in ("filter_ms", "tier1_ms", "tier2_ms", "per_level_ms",
                                                          "total_ms")},
                roofline=engine_roofline(ks, 1, prof_ms),
                parity="bit-exact counts+digests vs oracle, both paths, %d/%d" % (len(qs), len(qs)) if parity
                else "MISMATCH")


def ablation_variants(gsi):
    """(name, flags): the design as built, the per-level kernels as the
    paper describes them (the reference, 1.0), this design's departures, and
    the paper's ablations (Tables V-IX) on top of the per-level kernels."""
    PL = gsi.GSI_NO_FUSED | gsi.GSI_NO_LIST_FILTER
    return [("default", 0), ("per_level", PL), ("per_level+list_filter", gsi.GSI_NO_FUSED),
            ("level_first_edge", gsi.GSI_LEVEL_FIRST_EDGE), ("single_pass", gsi.GSI_SINGLE_PASS),
            ("per_level+cr_lookup", PL | gsi.GSI_ABL_CR),
            ("per_level+two_step_output", PL | gsi.GSI_ABL_TWO_STEP),
            ("per_level+unstaged_rows", PL | gsi.GSI_ABL_NO_STAGING),
            ("per_level+naive_set_ops", PL | gsi.GSI_ABL_NAIVE_SETOPS),
            ("per_level+row_per_wave", PL | gsi.GSI_ABL_ROW_PER_WAVE),
            ("per_level+row_per_wave+dup_removal", PL | gsi.GSI_ABL_ROW_PER_WAVE | gsi.GSI_ABL_DUP_REMOVAL),
            ("per_level+four_layer", PL | gsi.GSI_ABL_FOUR_LAYER),
            ("per_level+four_layer+dup_removal", PL | gsi.GSI_ABL_FOUR_LAYER | gsi.GSI_ABL_DUP_REMOVAL)]


PAPER_TABLES = {
    "per_level+cr_lookup": "Table VI: CR -> PCSR, 1.1-1.4x",
    "per_level+two_step_output": "Table V +PC: two-step output -> Prealloc-Combine, 1.2-2.0x",
    "per_level+unstaged_rows": "Table VII: write cache off -> on, 1.0-4.2x",
    "per_level+naive_set_ops": "Table V +SO: naive -> GPU-friendly set operations, 1.0-6.3x",
    "per_level+four_layer": "Table VIII: GSI -> +LB (4-layer balance), 1.0-3.4x",
    "per_level+four_layer+dup_removal": "Table VIII +DR: on top of +LB, 1.0-1.3x (Table IX: 3-23% fewer loads)",
}


def run_ablations(dg, qs, gold_q, passes):
    """Each variant over the queries, one at a time (rows written): one
    warm-up pass, then the best of `passes`; every variant's counts and
    digests must equal the oracle's."""
    import torch
    import paper_1906_03420_amd as gsi

    def run(flags):
        out = []
        t0 = time.perf_counter()
        for q in qs:
            r = dg.query(q, flags=flags)
            out.append((r.count, r.digest))
            r.free()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    res, ok = {}, True
    for name, flags in ablation_variants(gsi):
        run(flags)
        best = None
        for _ in range(max(1, passes)):
            dt, out = run(flags)
            best = dt if best is None else min(best, dt)
            ok &= all(c == x["count"] and [str(d[0]), str(d[1])] == x["digest"] for (c, d), x in zip(out, gold_q))
        res[name] = dict(ms_per_pass=best * 1e3)
    base = res["per_level"]["ms_per_pass"]
    for name in res:
        res[name]["vs_per_level"] = res[name]["ms_per_pass"] / base
        if name in PAPER_TABLES:
            res[name]["paper"] = PAPER_TABLES[name]
    return res, ok


def ablation_section(args, vl_t, s_t, d_t, l_t, g, qs, gold, arena):
    """The paper's ablations on the BA-1M single-query workload (100 queries):
    time per pass relative to the per-level kernels as the paper describes
    them (per_level = 1.0)."""
    import paper_1906_03420_amd as gsi
    ctx = gsi.Context(arena)
    dg = ctx.load_device(g.n, vl_t, s_t, d_t, l_t, gsi.GSI_GRAPH_KEEP_CR)
    res, ok = run_ablations(dg, qs, gold["queries"], args.steps)
    dg.free()
    ctx.close()
    return dict(workload="the BA-1M single-query workload (100 queries, rows written), best of %d passes"
                         % max(1, args.steps), variants=res,
                parity="bit-exact counts+digests vs oracle in every variant" if ok else "MISMATCH")


def ablation_section_c2(hx, arena, nq=8):
    """The same ablations on the R-MAT-23 queries whose joins are largest
    (the nq with the most embeddings below 10^8), where the join, not the
    per-query fixed cost, sets the time."""
    import numpy as np
    import torch
    import paper_1906_03420_amd as gsi
    gold = hx["gold"]["queries"]
    pick = sorted(range(len(gold)), key=lambda i: -gold[i]["count"])
    pick = [i for i in pick if gold[i]["count"] < 100_000_000][:nq]
    g = hx["g"]
    dev = torch.device("cuda:0")
    as_t = lambda a: torch.from_numpy(a.view(np.int32)).to(dev)
    ctx = gsi.Context(arena)
    dg = ctx.load_device(g.n, as_t(g.vlabel), as_t(g.src), as_t(g.dst), as_t(g.elabel), gsi.GSI_GRAPH_KEEP_CR)
    res, ok = run_ablations(dg, [hx["qs"][i] for i in pick], [gold[i] for i in pick], 1)
    dg.free()
    ctx.close()
    torch.cuda.empty_cache()
    return dict(workload="R-MAT-23, the %d queries with the most embeddings below 10^8 (indices %s; %d embeddings "
                         "per pass), rows written, best of 1 pass after a warm-up" %
                         (len(pick), [gold[i]["index"] for i in pick], sum(gold[i]["count"] for i in pick)),
                variants=res, parity="bit-exact counts+digests vs oracle in every variant" if ok else "MISMATCH")


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
    seq_lat = np.zeros(n)
    for j, r in enumerate(reqs0):
        tq = time.perf_counter()
        res = dg.query(pool[r])
        seq_lat[j] = time.perf_counter() - tq
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
    # the saturation run again with HIP events around every launch
    ctx = gsi.Context(arena, flags=gsi.GSI_CTX_PROFILE)
    dg = ctx.load_device(g.n, *tensors)
    ctx.kernel_stats_reset()
    tp = time.perf_counter()
    run(reqs0, None)
    prof_ms = (time.perf_counter() - tp) * 1e3
    dg.free()
    kst = [k for k in ctx.kernel_stats() if k["launches"]]
    ctx.close()
    del tensors
    ks = sorted(set(int(q.k) for q in pool))
    drawn = len(gold["queries"]) + len(gold.get("dropped", []))
    return dict(workload="R-MAT scale 22, %d vertices / %d edges, 64 vertex + 16 edge labels Zipf(1.1); pool of %d "
                         "queries (k %d-%d, tree / walk with a cycle / dense); %d requests per rate"
                         % (g.n, g.m, len(pool), ks[0], ks[-1], n),
                pool=dict(queries=len(gold["queries"]), indices_drawn=drawn, indices_dropped=drawn - len(gold["queries"]),
                          dropped_share=(drawn - len(gold["queries"])) / drawn if drawn else 0.0,
                          acceptance=gold.get("limits")),
                graph_gen_s=gen_s, one_at_a_time=dict(queries_per_s=n / t_seq,
                                                       embeddings_per_s=emb_of(reqs0) / t_seq,
                                                       p50_ms=float(np.percentile(seq_lat, 50) * 1e3),
                                                       p99_ms=float(np.percentile(seq_lat, 99) * 1e3),
                                                       what="submit -> answer ready on the device, one request "
                                                            "at a time, no queueing"),
                saturation=sat, speedup_vs_one_at_a_time=mu * t_seq / n, rates=rates,
                roofline=engine_roofline(kst, 1, prof_ms),
                parity=("bit-exact counts+digests vs oracle, every request (%d)" % (4 * n + n)) if total_bad == 0
                else "MISMATCH in %d answers" % total_bad)


def kernel_table(ks):
    return {k["name"]: dict(launches=k["launches"], ms=round(k["total_ms"], 3),
                            gbs=round(k["alg_bytes"] / (k["total_ms"] * 1e-3) / 1e9, 1) if k["total_ms"] else None)
            for k in ks}


def roofline_of(ks, names, steps, prof_ms):
    """Roofline line of the kernel among `names` with the largest summed
    device time: algorithmic bytes over its summed HIP-event durations.
    Entries "<kernel>@large" (launches of >= 16 MiB of algorithmic bytes,
    booked a second time) are read apart and kept out of the device total."""
    base = [k for k in ks if "@" not in k["name"]]
    dev_ms = sum(k["total_ms"] for k in base)
    cands = [k for k in base if k["name"] in names]
    if not cands:
        return None
    dom = max(cands, key=lambda k: k["total_ms"])
    achieved = dom["alg_bytes"] / (dom["total_ms"] * 1e-3) / 1e9
    large = {}
    for k in ks:
        if k["name"].endswith("@large") and k["name"].split("@")[0] in names and k["total_ms"]:
            gbs = k["alg_bytes"] / (k["total_ms"] * 1e-3) / 1e9
            large[k["name"]] = dict(launches=k["launches"], ms=round(k["total_ms"], 3), achieved_gbs=round(gbs, 1),
                                    frac=round(gbs / HBM_PEAK_GBS, 4))
    return dict(kernel=dom["name"], bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=achieved / HBM_PEAK_GBS, traffic=stored_traffic(dom["name"]),
                alg_bytes_per_launch=dom["alg_bytes"] / dom["launches"], launches=dom["launches"],
                avg_launch_us=dom["total_ms"] / dom["launches"] * 1e3,
                share_of_device_time=dom["total_ms"] / dev_ms if dev_ms else None,
                limiter=("latency: one 1024-thread workgroup runs every level of a small query"
                         if dom["name"] == "k_fused_levels" else "hbm"),
                measured="HIP events around every launch in %d profiled steps (%.1f ms/step with events)"
                         % (steps, prof_ms),
                large_launches=large)


ENGINE_KERNELS = ("k_filter", "k_wlocate", "k_wjoin", "k_wlink", "k_wdigest", "k_fused_batch<64>",
                  "k_fused_batch<256>", "k_fused_batch<1024>")


def engine_roofline(ks, steps, prof_ms):
    """Roofline of the batched / served path: the dominant kernel among the
    batched filter, the fused tiers and the level-synchronous engine, plus a
    line per engine kernel (algorithmic bytes over summed event time)."""
    line = roofline_of(ks, ENGINE_KERNELS, steps, prof_ms)
    per = {}
    for k in ks:
        if k["name"] in ENGINE_KERNELS and k["total_ms"]:
            gbs = k["alg_bytes"] / (k["total_ms"] * 1e-3) / 1e9
            per[k["name"]] = dict(launches=k["launches"], ms=round(k["total_ms"], 3), achieved_gbs=round(gbs, 1),
                                  frac=round(gbs / HBM_PEAK_GBS, 4))
    if line:
        line["per_kernel"] = per
    return line


def single_query_section(name, args, arena, steps, warmup, keep_tensors=False):
    """One workload on the single-query path: the graph is built once from
    its edge list in HBM (build time reported apart), then `steps` timed
    passes over its queries, one at a time, rows written to HBM; a pass
    that also copies each result's rows to host memory (D2H-inclusive
    latency); and the same passes again with HIP events around every launch
    for the per-kernel roofline."""
    import numpy as np
    import torch
    import paper_1906_03420_amd as gsi

    t = time.perf_counter()
    g, qs, gold = make_workload(name)
    gen_s = time.perf_counter() - t
    if args.queries and args.queries < len(qs):
        qs = qs[:args.queries]
        if gold:
            gold = dict(gold, queries=gold["queries"][:args.queries])
    progress("%s: graph and %d queries generated in %.1f s" % (name, len(qs), gen_s))
    dev = torch.device("cuda:0")
    as_t = lambda a: torch.from_numpy(a.view(np.int32)).to(dev)
    tens = (as_t(g.vlabel), as_t(g.src), as_t(g.dst), as_t(g.elabel))
    torch.cuda.synchronize()

    def build(ctx):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dg = ctx.load_device(g.n, *tens)
        torch.cuda.synchronize()
        return dg, time.perf_counter() - t0

    def step(dg, rows_to_host=False):
        lat, out = [], []
        for q in qs:
            tq = time.perf_counter()
            r = dg.query(q)
            if rows_to_host:
                r.rows()
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
    for _ in range(2):
        dg, bt = build(ctx)
        build_all.append(bt)
        dg.free()
    dg, bt = build(ctx)
    build_all.append(bt)
    parity_ok = None
    for _ in range(warmup):
        _, out = step(dg)
        if gold:
            parity_ok = matches(out) if parity_ok is None else (parity_ok and matches(out))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat_steps, outs = [], []
    for _ in range(steps):
        lat, out = step(dg)
        lat_steps.append(lat)
        outs.append(out)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    # answers checked after the timed steps
    emb = 0
    for out in outs:
        emb += sum(c for c, _ in out)
        if gold:
            parity_ok = matches(out) if parity_ok is None else (parity_ok and matches(out))
    # D2H-inclusive latency: the same queries with the rows copied to host
    lat_d2h, _ = step(dg, rows_to_host=True) if not args.no_d2h_pass else ([float("nan")] * len(qs), None)
    dg.free()
    ctx.close()

    ctx = gsi.Context(arena, flags=gsi.GSI_CTX_PROFILE)
    dg, _ = build(ctx)
    ctx.kernel_stats_reset()  # query kernels only
    tp = time.perf_counter()
    for _ in range(steps):
        step(dg)
    prof_ms = (time.perf_counter() - tp) / steps * 1e3
    dg.free()
    ks = [k for k in ctx.kernel_stats() if k["launches"]]
    ctx.close()
    torch.cuda.empty_cache()

    lat_all = np.array([x for lat in lat_steps for x in lat]) * 1e3
    med_lat_s = np.median(np.array(lat_steps), axis=0)
    d2h = np.array(lat_d2h) * 1e3
    res = dict(
        value=emb / total, ms_per_step=total / steps * 1e3,
        config=dict(workload=WORKLOAD_TEXT[name], name=name, queries=len(qs), path="single-query",
                    graph="resident; PCSR and signatures built before timing (build_ms)",
                    embeddings_per_step=emb // steps, rows="written to HBM (row-major, query-vertex order)"),
        queries_per_s=len(qs) * steps / total,
        latency_ms=dict(p50=float(np.percentile(lat_all, 50)), p99=float(np.percentile(lat_all, 99)),
                        max=float(lat_all.max()), what="submit -> count, digest and rows ready on the device"),
        latency_d2h_ms=dict(p50=float(np.percentile(d2h, 50)), p99=float(np.percentile(d2h, 99)),
                            max=float(d2h.max()), pass_ms=float(d2h.sum()),
                            what="submit -> rows copied to pageable host memory (one pass)"),
        build_ms=float(np.median(build_all) * 1e3), graph_gen_s=gen_s,
        parity=("bit-exact counts+digests vs oracle, %d/%d queries, every step" % (len(qs), len(qs))) if parity_ok
        else ("MISMATCH" if parity_ok is False else "no stored oracle values"),
        roofline=roofline_of(ks, HOT_KERNELS, steps, prof_ms),
        kernels=kernel_table(ks),
    )
    extra = dict(g=g, qs=qs, gold=gold, med_lat_s=med_lat_s)
    if keep_tensors:
        extra["tensors"] = tens
    return res, extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat23", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--queries", type=int, default=0, help="use only the first N queries of the workload (0: all)")
    ap.add_argument("--arena-gb", type=float, default=0.0, help="0: 160 GB for rmat23, 48 GB otherwise")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ba1m", action="store_true", help="skip the BA-1M single-query section")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-sequential comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-ablations", action="store_true", help="skip the ablation runs")
    ap.add_argument("--no-d2h-pass", action="store_true",
                    help="skip the pass that copies every result's rows to host memory (D2H-inclusive latency)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device copy of this size (a reference kernel for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (asked for %d)" % max(args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    gb = args.arena_gb or (160.0 if args.workload == "rmat23" else 48.0)
    head, hx = single_query_section(args.workload, args, int(gb * (1 << 30)), args.steps, args.warmup,
                                    keep_tensors=args.workload == "ba1m")
    progress("%s single-query path done: %.3g embeddings/s" % (args.workload, head["value"]))
    res = dict(metric=METRIC, value=head.pop("value"), unit="embeddings/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=head.pop("ms_per_step"), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="u32", data="synthetic", config=head.pop("config"))
    res.update(head)

    arena48 = int(48 * (1 << 30))
    bx = hx if args.workload == "ba1m" else None
    if not args.no_ba1m and args.workload != "ba1m":
        sec, bx = single_query_section("ba1m", args, arena48, args.steps, args.warmup, keep_tensors=True)
        res["ba1m"] = sec
        progress("ba1m single-query path done: %.3g embeddings/s" % sec["value"])
    if bx is not None and "tensors" in bx:
        vl_t, s_t, d_t, l_t = bx["tensors"]
        if not args.no_batched:
            res["batched"] = batched_section(args, vl_t, s_t, d_t, l_t, bx["g"], arena48)
            progress("batched section done")
        if not args.no_ablations and bx["gold"]:
            res["ablations"] = ablation_section(args, vl_t, s_t, d_t, l_t, bx["g"], bx["qs"], bx["gold"], arena48)
            progress("ablations done")
        del vl_t, s_t, d_t, l_t
        bx.pop("tensors")
        torch.cuda.empty_cache()
    if not args.no_ablations and args.workload == "rmat23" and hx["gold"]:
        res["ablations_rmat23"] = ablation_section_c2(hx, int(gb * (1 << 30)))
        progress("R-MAT-23 ablations done")
    if not args.no_serving:
        res["serving"] = serving_section(args, int(96 * (1 << 30)))
    if not args.no_cpu_baseline and hx["gold"]:
        res["cpu_baseline"] = cpu_baseline(hx["g"], hx["qs"], hx["gold"], hx["med_lat_s"])
        progress("cpu baseline done")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

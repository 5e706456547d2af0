"""Writes oracle counts and digests for the named workloads.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_golden.py er1k ba1m
    python tests/golden/make_golden.py --redigest er1k ba1m   (digests only)
The file is rewritten after every query and a rerun resumes after the last
query present, so a long workload can be written in several sittings; tests
check the queries the file holds.
Each query is accepted when the generator produces it and the oracle
finishes it within per-workload limits on embeddings and on search nodes
(each of the oracle's threads gets an equal share of the node cap, so the
thread count is recorded); otherwise it is redrawn with the next attempt
number and the rejection is logged in the output file.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as w  # noqa: E402

MAX_COUNT = {"er1k": 1_000_000_000, "ba1m": 1_000_000_000, "ba1m_batch": 1_000_000_000,
             "rmat23": 1_000_000_000, "rmat22_serve": 10_000_000}
MAX_NODES = {"er1k": 20_000_000_000, "ba1m": 20_000_000_000, "ba1m_batch": 4_000_000_000,
             "rmat23": 4_000_000_000, "rmat22_serve": 100_000_000}


# workloads whose acceptance records the oracle's thread count
NEW_STYLE = ("rmat23", "rmat22_serve")
# after this many rejected attempts an index is dropped (recorded in the file)
MAX_ATTEMPTS = {"rmat22_serve": 6}


def make(name: str, threads: int):
    c = w.CONFIGS[name]
    g = w.config_graph(name)
    og = oracle.OracleGraph(g)
    mk = w.QueryMaker(g)
    max_nodes, max_count = MAX_NODES[name], MAX_COUNT[name]
    limits = dict(max_count=max_count, max_nodes=max_nodes)
    if name in NEW_STYLE:
        limits["threads"] = threads
    if name in MAX_ATTEMPTS:
        limits["max_attempts"] = MAX_ATTEMPTS[name]
    out = dict(workload=name, n=g.n, m=g.m, limits=limits, queries=[], rejected=[])
    path = os.path.join(HERE, "%s.json" % name)
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("limits") == out["limits"] and old.get("n") == g.n and old.get("m") == g.m:
            out = old
    out.setdefault("dropped", [])

    def save():
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)

    start = 1 + max([x["index"] for x in out["queries"]] + out["dropped"], default=-1)
    for i in range(start, c["nq"]):
        attempt = 0
        while attempt < limits.get("max_attempts", 1 << 30):
            try:
                q = w.config_query(g, name, i, attempt=attempt, maker=mk)
            except RuntimeError:
                out["rejected"].append(dict(index=i, attempt=attempt, status="no walk"))
                attempt += 1
                continue
            t = time.time()
            r = og.match(q, threads=threads, tuples=False, max_count=max_count, max_nodes=max_nodes)
            dt = time.time() - t
            if r.status == oracle.OR_OK:
                break
            out["rejected"].append(dict(index=i, attempt=attempt, status=r.status))
            print(name, i, "rejected attempt", attempt, "status", r.status, round(dt, 1), flush=True)
            attempt += 1
        else:
            out["dropped"].append(i)
            print(name, i, "dropped", flush=True)
            save()
            continue
        out["queries"].append(dict(index=i, attempt=attempt, k=q.k, m=q.m, mode=q.mode, count=r.count,
                                   digest=[str(r.digest[0]), str(r.digest[1])], nodes=r.nodes,
                                   oracle_s=round(dt, 4)))
        print(name, i, q.k, r.count, round(dt, 1), flush=True)
        save()
    save()
    print("wrote", path)


def redigest(name: str, threads: int):
    """Recomputes the digest of every stored query (same index and accepted
    attempt, same limits) after a change of the digest's definition; the
    counts must not change."""
    path = os.path.join(HERE, "%s.json" % name)
    with open(path) as f:
        out = json.load(f)
    lim = out["limits"]
    g = w.config_graph(name)
    og = oracle.OracleGraph(g)
    mk = w.QueryMaker(g)
    for x in out["queries"]:
        q = w.config_query(g, name, x["index"], attempt=x["attempt"], maker=mk)
        r = og.match(q, threads=threads, tuples=False, max_count=lim["max_count"], max_nodes=lim["max_nodes"])
        if r.status != oracle.OR_OK or r.count != x["count"]:
            raise SystemExit("%s query %d: status %d count %d, stored %d" % (name, x["index"], r.status, r.count,
                                                                            x["count"]))
        x["digest"] = [str(r.digest[0]), str(r.digest[1])]
        print(name, x["index"], r.count, flush=True)
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1)
    os.replace(path + ".tmp", path)
    print("rewrote digests of", path)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--redigest":
        for nm in args[1:]:
            redigest(nm, threads=8)
    else:
        for nm in args or ["er1k", "ba1m"]:
            make(nm, threads=8)

"""Writes oracle counts and digests for the named workloads.

Calls only the CPU oracle and the seeded input generators.  Usage:
    python tests/golden/make_golden.py er1k ba1m
The file is rewritten after every query and a rerun resumes after the last
query present, so a long workload can be written in several sittings; tests
check the queries the file holds.
Each query is accepted when the generator produces it and the oracle
finishes it within deterministic limits (at most 10^9 embeddings and a
per-workload cap on search nodes); otherwise it is redrawn with the next
attempt number and the rejection is logged in the output file.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as w  # noqa: E402

MAX_COUNT = 1_000_000_000
MAX_NODES = {"er1k": 20_000_000_000, "ba1m": 20_000_000_000, "ba1m_batch": 4_000_000_000,
             "rmat23": 4_000_000_000}


def make(name: str, threads: int):
    c = w.CONFIGS[name]
    g = w.config_graph(name)
    og = oracle.OracleGraph(g)
    mk = w.QueryMaker(g)
    max_nodes = MAX_NODES[name]
    out = dict(workload=name, n=g.n, m=g.m, limits=dict(max_count=MAX_COUNT, max_nodes=max_nodes),
               queries=[], rejected=[])
    path = os.path.join(HERE, "%s.json" % name)
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("limits") == out["limits"] and old.get("n") == g.n and old.get("m") == g.m:
            out = old
    start = len(out["queries"])
    for i in range(start, c["nq"]):
        attempt = 0
        while True:
            try:
                q = w.config_query(g, name, i, attempt=attempt, maker=mk)
            except RuntimeError:
                out["rejected"].append(dict(index=i, attempt=attempt, status="no walk"))
                attempt += 1
                continue
            t = time.time()
            r = og.match(q, threads=threads, tuples=False, max_count=MAX_COUNT, max_nodes=max_nodes)
            dt = time.time() - t
            if r.status == oracle.OR_OK:
                break
            out["rejected"].append(dict(index=i, attempt=attempt, status=r.status))
            attempt += 1
        out["queries"].append(dict(index=i, attempt=attempt, k=q.k, m=q.m, mode=q.mode, count=r.count,
                                   digest=[str(r.digest[0]), str(r.digest[1])], nodes=r.nodes,
                                   oracle_s=round(dt, 4)))
        print(name, i, q.k, r.count, round(dt, 1), flush=True)
        with open(path + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(path + ".tmp", path)
    print("wrote", path)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["er1k", "ba1m"]:
        make(nm, threads=os.cpu_count() or 1)

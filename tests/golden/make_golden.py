"""Writes the stored expected values of the full-size parity tests.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
inputs (``paper_1606_07550_amd.inputs``); nothing is read from the GPU path.
The full-size workloads are too large for the oracle to run inside a GPU test
in seconds, so it runs once here and the results are committed:

* ``rmat24.json``: R-MAT scale 24 (edge factor 16, seed 24, the benchmark
  graph): edge count, triangle total, average clustering coefficient, and
  fingerprints of the per-node triangle counts and degrees; plus the exact
  T(v) and d(v) of the 16 highest-degree hubs, computed a second time by the
  oracle's per-node count straight from the raw pairs (a cross-check of the
  oracle's two code paths).
* ``batch4096.json``: the 4,096-graph batch (master seed 4096): per graph its
  node count, edge count, triangle total, average clustering coefficient and
  fingerprints of T and d.
* ``k4_pass.json``: 4-clique counts of the graphs whose largest out-degree
  falls in each range of the 4-clique pass kernels, and 5-clique counts of
  hub-and-core graphs whose centres reach the larger 5-clique kernel.
* ``serving_rmat22.json``: for 408 of the 20,000 BFS-ball queries on R-MAT
  22 (seed 22, query seed 2022): the 8 largest and 400 drawn uniformly
  (seed 4222), the induced subgraph's edge count, triangle total and
  average clustering coefficient.

A fingerprint of an integer array a[0..n) is the pair
(sum_v a[v] * (v + 1), sum_v a[v]^2 * (2v + 1)) modulo 2^64: a test compares
the GPU's per-node counts against the oracle's through it without storing
them (314 MB for the batch).

Usage: python tests/golden/make_golden.py [rmat24|batch|k4|serving|all]
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def fingerprint(a):
    """(sum a[v](v+1), sum a[v]^2 (2v+1)) mod 2^64 of an integer array."""
    a = np.ascontiguousarray(a).astype(np.uint64)
    v = np.arange(a.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        h1 = int((a * (v + np.uint64(1))).sum(dtype=np.uint64))
        h2 = int((a * a * (np.uint64(2) * v + np.uint64(1))).sum(dtype=np.uint64))
    return [h1, h2]


def rmat24():
    import oracle
    from paper_1606_07550_amd import inputs as I
    t0 = time.time()
    n, s, d = I.rmat(24, 16, seed=24)
    print(f"rmat24 generated in {time.time() - t0:.1f}s", flush=True)
    t0 = time.time()
    ref = oracle.count(n, s, d, order=1)
    print(f"rmat24 oracle count {time.time() - t0:.1f}s total={ref['total']}", flush=True)
    deg = ref["deg"]
    hubs = np.argsort(-deg, kind="stable")[:16].astype(np.int32)
    t0 = time.time()
    samp = oracle.sampled(n, s, d, np.sort(hubs))
    print(f"rmat24 sampled hubs {time.time() - t0:.1f}s", flush=True)
    hs = np.sort(hubs)
    assert np.array_equal(samp["deg"], deg[hs]), "oracle paths disagree on hub degrees"
    assert np.array_equal(samp["T"], ref["T"][hs]), "oracle paths disagree on hub triangles"
    out = {
        "_source": "CPU oracle (oracle/tricc_oracle.c, node iterator with (d, id) rank) on R-MAT scale 24, "
                   "edge factor 16, seed 24, abcd .57/.19/.19/.05, noise 0.1, permuted; written by "
                   "tests/golden/make_golden.py",
        "n": int(n), "m_raw": int(s.size), "m": ref["m"], "total": ref["total"],
        "avg_hex": float(ref["avg"]).hex(),
        "T_fp": fingerprint(ref["T"]), "deg_fp": fingerprint(deg),
        "hubs": [{"node": int(v), "deg": int(deg[v]), "T": int(ref["T"][v])} for v in hs],
    }
    with open(os.path.join(HERE, "rmat24.json"), "w") as f:
        json.dump(out, f, indent=1)


def batch():
    import oracle
    from paper_1606_07550_amd import inputs as I
    G = 4096
    bt = I.batch(G, 4096)
    no, eo = bt["node_off"], bt["edge_off"]

    def one(g):
        a, e = int(no[g]), int(no[g + 1])
        e0, e1 = int(eo[g]), int(eo[g + 1])
        r = oracle.count(e - a, bt["src"][e0:e1], bt["dst"][e0:e1], threads=1)
        return {"n": e - a, "m": r["m"], "total": r["total"], "avg_hex": float(r["avg"]).hex(),
                "T_fp": fingerprint(r["T"]), "deg_fp": fingerprint(r["deg"])}

    t0 = time.time()
    order = np.argsort(-np.diff(eo))  # largest first
    res = [None] * G
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 1) as ex:
        for g, r in zip(order, ex.map(one, order)):
            res[int(g)] = r
    print(f"batch oracle {time.time() - t0:.1f}s", flush=True)
    out = {
        "_source": "CPU oracle (oracle/tricc_oracle.c) on each graph of the 4,096-graph batch (master seed "
                   "4096, n log-uniform in [64, 65536], BA or ER by a fair coin); written by "
                   "tests/golden/make_golden.py",
        "graphs": res,
    }
    with open(os.path.join(HERE, "batch4096.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


def k4():
    import oracle
    from paper_1606_07550_amd.inputs import fixtures as F
    out = {"_source": "CPU oracle (oracle_k4) on the seeded hub-and-core graphs of "
                      "paper_1606_07550_amd.inputs.fixtures.k4_core; written by tests/golden/make_golden.py",
           "graphs": []}
    for core, centres, avg_deg, seed in F.K4_CORE_CASES:
        n, s, d = F.k4_core(core, centres, avg_deg, seed)
        t0 = time.time()
        c = oracle.k4(n, s, d, order=1)
        print(f"k4 core={core} centres={centres}: {c} in {time.time() - t0:.1f}s", flush=True)
        out["graphs"].append({"core": core, "centres": centres, "avg_deg": avg_deg, "seed": seed, "n": int(n),
                              "k4": c})
    out["k5_graphs"] = []
    for core, centres, avg_deg, seed in F.K5_CORE_CASES:
        n, s, d = F.k4_core(core, centres, avg_deg, seed)
        t0 = time.time()
        c = oracle.k5(n, s, d, order=1)
        print(f"k5 core={core} centres={centres}: {c} in {time.time() - t0:.1f}s", flush=True)
        out["k5_graphs"].append({"core": core, "centres": centres, "avg_deg": avg_deg, "seed": seed, "n": int(n),
                                 "k5": c})
    with open(os.path.join(HERE, "k4_pass.json"), "w") as f:
        json.dump(out, f, indent=1)


def serving_picks(sizes):
    """The queries the stored serving results cover: the 8 largest and 400
    drawn uniformly (seed 4222), ascending."""
    rng = np.random.default_rng(4222)
    return np.unique(np.concatenate([np.argsort(sizes, kind="stable")[-8:],
                                     rng.choice(sizes.size, size=400, replace=False)]))


def serving():
    import oracle
    from paper_1606_07550_amd import inputs as I
    n, s, d = I.rmat(22, 16, seed=22)
    Q = 20000
    off, nodes, _ = I.bfs_queries(n, s, d, Q, seed=2022)
    picks = serving_picks(np.diff(off))

    def one(q):
        S = nodes[off[q]:off[q + 1]]
        r = oracle.induced(n, s, d, S, threads=1)
        return {"q": int(q), "k": int(S.size), "m": r["m"], "total": r["total"], "avg_hex": float(r["avg"]).hex()}

    t0 = time.time()
    order = sorted(picks.tolist(), key=lambda q: -(off[q + 1] - off[q]))  # largest first
    res = {}
    with ThreadPoolExecutor(max_workers=os.cpu_count() or 1) as ex:
        for q, r in zip(order, ex.map(one, order)):
            res[q] = r
    print(f"serving oracle {time.time() - t0:.1f}s for {len(order)} queries", flush=True)
    out = {
        "_source": "CPU oracle (oracle_induced) on R-MAT scale 22 (edge factor 16, seed 22, permuted) for the "
                   "BFS-ball queries of paper_1606_07550_amd.inputs.bfs_queries (20,000 queries, seed 2022) "
                   "listed by tests/golden/make_golden.py serving_picks; written by tests/golden/make_golden.py",
        "queries": [res[q] for q in sorted(res)],
    }
    with open(os.path.join(HERE, "serving_rmat22.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("k4", "all"):
        k4()
    if what in ("batch", "all"):
        batch()
    if what in ("rmat24", "all"):
        rmat24()
    if what in ("serving", "all"):
        serving()

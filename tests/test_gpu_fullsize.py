"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (its cached tuning, or the default):
- R-MAT 20: every node against the oracle;
- R-MAT 24 (the benchmark graph): every node against the oracle through the
  stored oracle results (tests/golden/rmat24.json: edge count, total,
  average, fingerprints of T(v) and d(v), and the 16 largest hubs' exact
  T(v) and d(v)), the total from the kernels' own counters, plus identities
  that hold at any size (T(v) <= C(d(v), 2), CC(v) from T(v) and d(v));
- the 4,096-graph batch: every graph against the stored oracle results
  (tests/golden/batch4096.json), and the batch total from the kernels' own
  counters against the sum of the graph totals;
- serving on R-MAT 22: sampled queries (the largest and random ones) of the
  20,000-query trace against the oracle's induced-subgraph count;
- edge-existence tests on G(n=10M, m=100M): every input pair positive, 2M
  sampled queries against the oracle;
- core numbers on R-MAT 22, every node against the oracle.
"""
import json
import os

import time

import numpy as np
import pytest
import torch

import oracle
import paper_1606_07550_amd as P
from paper_1606_07550_amd import autotune
from paper_1606_07550_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CC_RTOL = 1e-6
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def fingerprint(a):
    """(sum a[v](v+1), sum a[v]^2 (2v+1)) mod 2^64, as tests/golden/make_golden.py
    stores it for the oracle's arrays."""
    a = np.ascontiguousarray(a).astype(np.uint64)
    v = np.arange(a.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return [int((a * (v + np.uint64(1))).sum(dtype=np.uint64)),
                int((a * a * (np.uint64(2) * v + np.uint64(1))).sum(dtype=np.uint64))]


def say(msg):
    print(f"[fullsize] {msg}", flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def single_tuning(workload):
    rec = autotune.lookup(workload)
    return rec["tuning"] if rec else None


def run_single(n, s, d, workload):
    g = P.Graph(n, dev(s), dev(d), tuning=single_tuning(workload))
    o = g.count()
    torch.cuda.synchronize()
    return g, {
        "T": o["T"].cpu().numpy().view(np.uint64),
        "cc": o["cc"].cpu().numpy(),
        "total": int(o["total"].cpu().numpy().view(np.uint64)[0]),
        "avg": float(o["avg"].item()),
        "deg": g.arrays()["deg"].cpu().numpy(),
        "check": g.count_check(),
    }


def check_identities(r):
    T, deg = r["T"], r["deg"].astype(np.int64)
    # the total comes from the intersection kernels' own counters, not from T
    assert int(T.sum(dtype=np.uint64)) == 3 * r["total"]
    assert r["check"] == (r["total"], int(T.sum(dtype=np.uint64)))
    assert np.all(T.astype(np.float64) <= deg * (deg - 1) / 2)
    dd = deg.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(deg >= 2, 2.0 * T.astype(np.float64) / (dd * (dd - 1.0)), 0.0)
    np.testing.assert_array_equal(r["cc"], ratio.astype(np.float32))  # one rounding of the FP64 ratio
    assert abs(r["avg"] - ratio.mean()) <= 1e-12 * max(abs(ratio.mean()), 1e-300)


def test_rmat20_every_node():
    n, s, d = I.rmat(20, 16, seed=20)
    say(f"rmat20 n={n} m_raw={s.size}")
    _, r = run_single(n, s, d, "rmat20")
    ref = oracle.count(n, s, d, order=1)
    np.testing.assert_array_equal(r["T"], ref["T"])
    assert r["total"] == ref["total"]
    np.testing.assert_allclose(r["cc"].astype(np.float64), ref["cc"], rtol=CC_RTOL, atol=0)
    assert np.array_equal(r["cc"] == 0, ref["cc"] == 0)
    assert abs(r["avg"] - ref["avg"]) <= CC_RTOL * abs(ref["avg"])
    check_identities(r)


def test_rmat24_every_node_against_stored_oracle():
    ref = golden("rmat24.json")
    n, s, d = I.rmat(24, 16, seed=24)
    assert (n, s.size) == (ref["n"], ref["m_raw"])
    say(f"rmat24 n={n} m_raw={s.size}")
    g, r = run_single(n, s, d, "rmat24")
    say(f"rmat24 total={r['total']} m={g.info['m']}")
    assert g.info["m"] == ref["m"]
    assert r["total"] == ref["total"]
    assert fingerprint(r["deg"]) == ref["deg_fp"]
    assert fingerprint(r["T"]) == ref["T_fp"]
    assert abs(r["avg"] - float.fromhex(ref["avg_hex"])) <= CC_RTOL * float.fromhex(ref["avg_hex"])
    for h in ref["hubs"]:  # the largest hubs, whose T(v) take the most atomics
        assert (int(r["deg"][h["node"]]), int(r["T"][h["node"]])) == (h["deg"], h["T"]), h
    check_identities(r)


def test_batch_4096_every_graph_against_stored_oracle():
    G = 4096
    ref = golden("batch4096.json")["graphs"]
    bt = I.batch(G, 4096)
    node_off, edge_off = bt["node_off"], bt["edge_off"]
    assert len(ref) == G and [x["n"] for x in ref] == np.diff(node_off).tolist()
    say(f"batch G={G} nodes={node_off[-1]} pairs={edge_off[-1]}")
    b = P.Batch(node_off, edge_off, dev(bt["src"]), dev(bt["dst"]),
                tuning=autotune.default_or_cached_batch(f"batched-{G}"))
    b.plan()
    b.run()
    torch.cuda.synchronize()
    T = b.out["T"].cpu().numpy().view(np.uint64)
    cc = b.out["cc"].cpu().numpy()
    gtri = b.out["graph_tri"].cpu().numpy().view(np.uint64)
    gavg = b.out["graph_avg"].cpu().numpy()
    btri = int(b.out["batch_tri"].cpu().numpy().view(np.uint64)[0])
    deg = b.graph_arrays()["deg"].cpu().numpy()
    assert btri == int(gtri.sum(dtype=np.uint64)) == sum(x["total"] for x in ref)
    for gi in range(G):
        a, e = int(node_off[gi]), int(node_off[gi + 1])
        x = ref[gi]
        assert int(gtri[gi]) == x["total"], gi
        assert fingerprint(T[a:e]) == x["T_fp"], gi
        assert fingerprint(deg[a:e]) == x["deg_fp"], gi
        avg = float.fromhex(x["avg_hex"])
        assert abs(gavg[gi] - avg) <= CC_RTOL * abs(avg), gi
    # CC(v) from the (now verified) T(v) and d(v), rounded once from FP64
    dd = deg.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(deg >= 2, 2.0 * T.astype(np.float64) / (dd * (dd - 1.0)), 0.0)
    np.testing.assert_array_equal(cc, ratio.astype(np.float32))
    say(f"batch: all {G} graphs against the stored oracle results")

def test_edge_queries_er_10m_100m_sampled():
    """The benchmark's edge-existence configuration, G(n=10M, m=100M) with
    random queries: every input pair tests positive, and 1M random queries
    plus 1M input pairs (reversed) match the oracle."""
    n, m = 10_000_000, 100_000_000
    s, d = I.er(n, m, 2016)
    say(f"edge queries: G(n={n}, m={m})")
    g = P.Graph(n, dev(s), dev(d))
    pos = g.has_edges(dev(s), dev(d))
    assert bool(pos.all().item())
    rng = np.random.default_rng(2020)
    k = 1_000_000
    e = rng.integers(0, m, k)
    qu = np.concatenate([rng.integers(0, n, k), d[e]]).astype(np.int32)
    qv = np.concatenate([rng.integers(0, n, k), s[e]]).astype(np.int32)
    got = g.has_edges(dev(qu), dev(qv)).cpu().numpy()
    say("edge queries: oracle on 2M queries ...")
    np.testing.assert_array_equal(got, oracle.has_edges(n, s, d, qu, qv))
    say("edge queries: done")


def test_core_numbers_rmat22():
    """Every node's core number on R-MAT 22 against the oracle's bucket
    algorithm, and the 3-core (stop level 3)."""
    n, s, d = I.rmat(22, 16, seed=22)
    say(f"core numbers: rmat22 n={n}")
    g = P.Graph(n, dev(s), dev(d))
    c, mx = g.core()
    c3, _ = g.core(3)
    got, got3 = c.cpu().numpy(), c3.cpu().numpy()
    say("core numbers: oracle ...")
    ref = oracle.core(n, s, d)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got3, np.minimum(ref, 3))
    assert mx == ref.max()
    say(f"core numbers: max core {mx}")


def test_serving_rmat22_stored_queries():
    """408 of the 20,000 queries (the 8 largest, 400 drawn uniformly) against
    the stored oracle results, served as one mix."""
    ref = golden("serving_rmat22.json")["queries"]
    n, s, d = I.rmat(22, 16, seed=22)
    Q = 20000
    off, nodes, _ = I.bfs_queries(n, s, d, Q, seed=2022)
    say(f"serving resident n={n}, {Q} queries, {off[-1]} query nodes; {len(ref)} stored results")
    g = P.Graph(n, dev(s), dev(d))
    srv = P.Server(g, int(24e9), slots=3, max_batch_queries=256)
    srv.set_tuning({"merge_limit": 16, "wave_limit": 64, "persist_variant": 2, "blocks_per_cu": 0})
    pending = [x["q"] for x in ref]
    res = {}
    while pending or len(res) < len(ref):
        while pending:
            q = pending[0]
            if srv.submit(q, nodes[off[q]:off[q + 1]]) != 0:
                break  # admission full: collect results first
            pending.pop(0)
        got = srv.poll()
        for r in got:
            res[r["qid"]] = r
        if pending and not srv.stats()["in_flight"] and not srv.stats()["waiting"]:
            raise AssertionError("a query is refused with nothing in flight")
        if not got:
            time.sleep(0.002)
    srv.drain()
    for r in srv.poll():
        res[r["qid"]] = r
    assert len(res) == len(ref)
    for x in ref:
        r = res[x["q"]]
        assert r["status"] == 0 and r["k"] == x["k"], x["q"]
        assert r["triangles"] == x["total"], x["q"]
        assert r["m"] == x["m"], x["q"]
        avg = float.fromhex(x["avg_hex"])
        assert abs(r["avg_cc"] - avg) <= CC_RTOL * abs(avg), x["q"]
    srv.close()
    say(f"serving: {len(ref)} queries against the stored oracle results (largest k = {max(x['k'] for x in ref)})")

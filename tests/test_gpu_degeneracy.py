"""GPU checks of the degeneracy ordering (tricc_graph_degeneracy) and of
re-orientation by a key (tricc_graph_reorient).

The ordering itself is not unique (nodes peeled in one round may be taken in
any order), so it is checked for what makes it a degeneracy ordering: under
the orientation by (order, id) every node's out-degree is at most its core
number, and the core numbers equal the oracle's. The counts on a re-oriented
DAG are unique and are compared with the oracle exactly (triangles, T(v),
clustering coefficients, 4-cliques), also for an arbitrary random key, and
after re-orienting back to the degree order."""
import numpy as np
import pytest
import torch

import oracle
import paper_1606_07550_amd as P
from paper_1606_07550_amd import inputs as I
from paper_1606_07550_amd.inputs import fixtures as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def simple_edges(n, s, d):
    a = np.minimum(s, d).astype(np.int64)
    b = np.maximum(s, d).astype(np.int64)
    keep = a != b
    key = np.unique(a[keep] * n + b[keep])
    return key // n, key % n


def check_dag(g, n, s, d, key):
    """The DAG holds every simple edge once, oriented from the lower to the
    higher (key, id), each out-list ascending."""
    u, v = simple_edges(n, s, d)
    k = key.astype(np.int64)
    lo = np.where((k[u] < k[v]) | ((k[u] == k[v]) & (u < v)), u, v)
    hi = np.where(lo == u, v, u)
    A = g.arrays()
    doff = A["doff"].cpu().numpy()
    dcol = A["dcol"].cpu().numpy()
    dplus = np.diff(doff)
    np.testing.assert_array_equal(dplus, np.bincount(lo, minlength=n))
    src = np.repeat(np.arange(n), dplus)
    got = np.sort(src.astype(np.int64) * n + dcol)
    np.testing.assert_array_equal(got, np.sort(lo * n + hi))
    if dcol.size:
        same = src[1:] == src[:-1]
        assert np.all(dcol[1:][same] > dcol[:-1][same]), "out-lists not ascending"
    assert g.info["max_outdeg"] == (dplus.max() if n else 0)
    return dplus


def counts(g):
    o = g.count()
    k4 = int(g.count_k4().cpu().numpy().view(np.uint64)[0])
    torch.cuda.synchronize()
    return (o["T"].cpu().numpy().view(np.uint64), int(o["total"].cpu().numpy().view(np.uint64)[0]),
            o["cc"].cpu().numpy(), float(o["avg"].item()), k4)


CASES = {
    "rmat14": lambda: I.rmat(14, 16, seed=61),
    "rmat17": lambda: I.rmat(17, 16, seed=62),
    "ba": lambda: (30000, *I.ba(30000, 8, 63)),
    "families": lambda: F.disjoint_union(F.complete(30), F.wheel(25), F.ring_lattice(60, 6), F.windmill(5),
                                         F.grid(6, 7), F.star(40)),
    "empty": lambda: (5, np.zeros(0, np.int32), np.zeros(0, np.int32)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_degeneracy_order_and_counts(name):
    n, s, d = CASES[name]()
    print(f"[degeneracy] {name} n={n} m_raw={len(s)}", flush=True)
    ref = oracle.count(n, s, d, order=1)
    ref_k4 = oracle.k4(n, s, d, order=1)
    ref_core = oracle.core(n, s, d)
    g = P.Graph(n, dev(s), dev(d))
    base_max = g.info["max_outdeg"]
    order, core, dg = g.degeneracy()
    order, core = order.cpu().numpy(), core.cpu().numpy()
    np.testing.assert_array_equal(core, ref_core)
    assert dg == (int(ref_core.max()) if n else 0)
    g.reorient(torch.from_numpy(order).to(DEV))
    dplus = check_dag(g, n, s, d, order)
    assert np.all(dplus <= core), "an out-degree above the core number"
    assert g.info["max_outdeg"] <= dg <= max(base_max, dg)
    T, tot, cc, avg, k4 = counts(g)
    np.testing.assert_array_equal(T, ref["T"])
    assert tot == ref["total"] and k4 == ref_k4
    np.testing.assert_allclose(cc.astype(np.float64), ref["cc"], rtol=1e-6, atol=0)
    assert abs(avg - ref["avg"]) <= 1e-6 * abs(ref["avg"])
    assert g.count_check() == (tot, int(T.sum(dtype=np.uint64)))
    # back to the degree order
    g.reorient(None)
    assert g.info["max_outdeg"] == base_max
    deg = g.arrays()["deg"].cpu().numpy()
    check_dag(g, n, s, d, deg)
    T2, tot2, _, _, k42 = counts(g)
    np.testing.assert_array_equal(T2, ref["T"])
    assert tot2 == ref["total"] and k42 == ref_k4


def test_reorient_by_random_key():
    n, s, d = I.rmat(15, 16, seed=64)
    ref = oracle.count(n, s, d, order=1)
    g = P.Graph(n, dev(s), dev(d))
    key = np.random.default_rng(65).integers(0, 1 << 20, n).astype(np.int32)
    g.reorient(torch.from_numpy(key).to(DEV))
    check_dag(g, n, s, d, key)
    if g.info["max_outdeg"] <= 4096:
        T, tot, _, _, k4 = counts(g)
        assert k4 == oracle.k4(n, s, d, order=1)
    else:
        o = g.count()
        torch.cuda.synchronize()
        T, tot = o["T"].cpu().numpy().view(np.uint64), int(o["total"].cpu().numpy().view(np.uint64)[0])
    np.testing.assert_array_equal(T, ref["T"])
    assert tot == ref["total"]

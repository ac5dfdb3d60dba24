"""Pins of the CPU oracle against things other than itself: hand-worked
examples, brute force over all node triples, dense and sparse linear algebra,
networkx, closed forms of regular families, invariants, and planted mistakes.
"""
import itertools
import json
import os
import shutil
import subprocess
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1606_07550_amd import inputs as I
from paper_1606_07550_amd.inputs import fixtures as F

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# independent references (test code only)

def adjacency(n, s, d):
    A = np.zeros((n, n), dtype=np.int64)
    A[s, d] = 1
    A[d, s] = 1
    np.fill_diagonal(A, 0)
    return A


def brute_force(n, s, d):
    """All node triples, pairwise adjacency checked directly; exact fractions."""
    A = adjacency(n, s, d).astype(bool)
    T = np.zeros(n, dtype=np.int64)
    total = 0
    for a, b, c in itertools.combinations(range(n), 3):
        if A[a, b] and A[b, c] and A[a, c]:
            total += 1
            T[a] += 1
            T[b] += 1
            T[c] += 1
    deg = A.sum(1)
    cc = [Fraction(int(2 * T[v]), int(deg[v] * (deg[v] - 1))) if deg[v] >= 2 else Fraction(0) for v in range(n)]
    avg = sum(cc, Fraction(0)) / n if n else Fraction(0)
    return T, total, cc, avg, deg


def assert_matches(r, T, total, cc=None, avg=None, rel=1e-12):
    np.testing.assert_array_equal(r["T"].astype(np.int64), np.asarray(T, dtype=np.int64))
    assert r["total"] == total
    if cc is not None:
        ref = np.array([float(c) for c in cc])
        np.testing.assert_allclose(r["cc"], ref, rtol=rel, atol=0)
        assert np.all((ref == 0) == (r["cc"] == 0))
    if avg is not None:
        assert r["avg"] == pytest.approx(float(avg), rel=rel, abs=1e-300)


# ---------------------------------------------------------------------------

def test_golden_small_graphs():
    with open(os.path.join(HERE, "golden", "small_graphs.json")) as f:
        data = json.load(f)
    for g in data["graphs"]:
        e = np.array(g["edges"], dtype=np.int32).reshape(-1, 2)
        for order in (0, 1):
            r = oracle.count(g["n"], e[:, 0], e[:, 1], order=order)
            assert r["total"] == g["total"], g["name"]
            np.testing.assert_array_equal(r["T"], np.array(g["T"], dtype=np.uint64), err_msg=g["name"])
            np.testing.assert_allclose(r["cc"], [float(Fraction(c)) for c in g["cc"]], rtol=1e-15, err_msg=g["name"])
            assert r["avg"] == pytest.approx(float(Fraction(g["avg"])), rel=1e-15), g["name"]


def _small_cases():
    out = []
    for n, m, seed in [(12, 30, 1), (20, 60, 2), (30, 200, 3), (40, 300, 4), (25, 150, 5)]:
        s, d = I.er(n, m, seed)
        out.append((f"er{n}_{m}", n, s, d))
    s, d = I.ba(30, 3, 7)
    out.append(("ba30", 30, s, d))
    n, s, d = I.rmat(5, 8, seed=9)  # 256 pairs on 32 nodes: duplicates and loops included
    out.append(("rmat5", n, s, d))
    n, s, d = F.messy(*F.complete(9), seed=3)
    out.append(("messyK9", n, s, d))
    return out


@pytest.mark.parametrize("name,n,s,d", _small_cases(), ids=[c[0] for c in _small_cases()])
@pytest.mark.parametrize("order", [0, 1])
def test_brute_force(name, n, s, d, order):
    T, total, cc, avg, deg = brute_force(n, s, d)
    r = oracle.count(n, s, d, order=order)
    assert_matches(r, T, total, cc, avg)
    np.testing.assert_array_equal(r["deg"], deg)


@pytest.mark.parametrize("case", ["er", "ba", "rmat"])
def test_dense_cube(case):
    """T(v) = (A^3)_vv / 2 and T = trace(A^3) / 6 in exact int64 arithmetic."""
    if case == "er":
        n = 1500
        s, d = I.er(n, 20000, 11)
    elif case == "ba":
        n = 1000
        s, d = I.ba(n, 8, 12)
    else:
        n, s, d = I.rmat(10, 16, seed=13)
    A = adjacency(n, s, d)
    A3d = np.einsum("ij,ji->i", A @ A, A)
    assert np.all(A3d % 2 == 0)
    r = oracle.count(n, s, d, order=1)
    np.testing.assert_array_equal(r["T"].astype(np.int64), A3d // 2)
    assert r["total"] * 6 == int(A3d.sum())
    deg = A.sum(1)
    np.testing.assert_array_equal(r["deg"], deg)
    m = int(A.sum()) // 2
    assert r["m"] == m


def test_sparse_er_config():
    """G(n=10^4, m=10^5): T(v) = 1/2 sum_u A_vu (A^2)_vu with scipy (int64)."""
    n, m = 10_000, 100_000
    s, d = I.er(n, m, 1)
    A = sp.coo_matrix((np.ones(m, np.int64), (s, d)), shape=(n, n)).tocsr()
    A = ((A + A.T) > 0).astype(np.int64)
    A.setdiag(0)
    A.eliminate_zeros()
    Tref = np.asarray(A.multiply(A @ A).sum(axis=1)).ravel() // 2
    for order in (0, 1):
        r = oracle.count(n, s, d, order=order)
        np.testing.assert_array_equal(r["T"].astype(np.int64), Tref)
        assert r["m"] == m
    # sanity only: E[T] = C(n,3) p^3 with p = m / C(n,2), about 1333
    assert 1000 < r["total"] < 1700


@pytest.mark.parametrize("case", ["er", "ba", "rmat"])
def test_networkx(case):
    if case == "er":
        n = 2000
        s, d = I.er(n, 20000, 21)
    elif case == "ba":
        n = 3000
        s, d = I.ba(n, 5, 22)
    else:
        n, s, d = I.rmat(11, 8, seed=23)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(s, d) if a != b)
    tri = nx.triangles(G)
    clu = nx.clustering(G)
    r = oracle.count(n, s, d, order=1)
    np.testing.assert_array_equal(r["T"], np.array([tri[v] for v in range(n)], dtype=np.uint64))
    np.testing.assert_allclose(r["cc"], [clu[v] for v in range(n)], rtol=1e-12, atol=0)
    assert r["avg"] == pytest.approx(nx.average_clustering(G), rel=1e-12)
    assert r["total"] == sum(tri.values()) // 3


def _comb(a, b):
    from math import comb
    return comb(a, b)


def test_closed_forms():
    for n in range(1, 13):
        r = oracle.count(*F.complete(n))
        assert r["total"] == _comb(n, 3)
        assert np.all(r["T"] == _comb(n - 1, 2))
        if n >= 3:
            assert np.all(r["cc"] == 1.0) and r["avg"] == 1.0
    for n in range(4, 30):
        r = oracle.count(*F.ring(n))
        assert r["total"] == 0 and r["avg"] == 0.0
    r = oracle.count(*F.ring(3))
    assert r["total"] == 1 and np.all(r["cc"] == 1.0)
    zero_cases = [F.star(50), F.path(40), F.random_tree(300, 5), F.grid(13, 17),
                  F.complete_bipartite(7, 9), F.random_bipartite(60, 40, 0.3, 6)]
    for g in zero_cases:
        r = oracle.count(*g)
        assert r["total"] == 0 and not np.any(r["T"]) and not np.any(r["cc"]) and r["avg"] == 0.0
    for rim in range(4, 25):
        r = oracle.count(*F.wheel(rim))
        assert r["total"] == rim
        assert r["T"][0] == rim and np.all(r["T"][1:] == 2)
        assert r["cc"][0] == pytest.approx(2.0 / (rim - 1), rel=1e-15)
        np.testing.assert_allclose(r["cc"][1:], 2.0 / 3.0, rtol=1e-15)
    for k in range(1, 20):
        r = oracle.count(*F.windmill(k))
        assert r["total"] == k
        assert r["cc"][0] == pytest.approx(1.0 / (2 * k - 1), rel=1e-15)
        assert np.all(r["cc"][1:] == 1.0)
    for K in (2, 4, 6, 8, 10):
        for n in (3 * K // 2 + 1, 3 * K // 2 + 5, 100):
            r = oracle.count(*F.ring_lattice(n, K))
            assert np.all(r["T"] == 3 * K * (K - 2) // 8), (n, K)
            np.testing.assert_allclose(r["cc"], 3.0 * (K - 2) / (4.0 * (K - 1)), rtol=1e-15)


def test_invariants():
    n, s, d = I.rmat(12, 16, seed=31)
    base = oracle.count(n, s, d, order=1)
    assert int(base["T"].sum()) == 3 * base["total"]
    deg = base["deg"]
    assert np.all(base["T"] <= deg * (deg - 1) // 2)
    assert np.all((base["cc"] >= 0) & (base["cc"] <= 1))
    assert base["avg"] == pytest.approx(base["cc"].mean(), rel=1e-13)
    # noisy input of the same simple graph
    r = oracle.count(*F.messy(n, s, d, seed=32), order=0)
    np.testing.assert_array_equal(r["T"], base["T"])
    assert r["avg"] == pytest.approx(base["avg"], rel=1e-13)
    # relabelling permutes the per-node values
    n2, s2, d2, perm = F.relabel(n, s, d, seed=33)
    r = oracle.count(n2, s2, d2, order=1)
    np.testing.assert_array_equal(r["T"][perm], base["T"])
    np.testing.assert_array_equal(r["cc"][perm], base["cc"])
    # disjoint union: per-node values unchanged, totals add
    g2 = F.wheel(9)
    nu, su, du = F.disjoint_union((n, s, d), g2)
    r = oracle.count(nu, su, du, order=1)
    np.testing.assert_array_equal(r["T"][:n], base["T"])
    assert r["total"] == base["total"] + 9


@pytest.mark.parametrize("case", ["er", "rmat", "ba"])
def test_orders_agree(case):
    if case == "er":
        n = 10_000
        s, d = I.er(n, 100_000, 1)
    elif case == "rmat":
        n, s, d = I.rmat(14, 16, seed=41)
    else:
        n = 20_000
        s, d = I.ba(n, 6, 42)
    a = oracle.count(n, s, d, order=0)
    b = oracle.count(n, s, d, order=1)
    np.testing.assert_array_equal(a["T"], b["T"])
    np.testing.assert_array_equal(a["cc"], b["cc"])
    assert a["total"] == b["total"] and a["avg"] == b["avg"]


def test_induced():
    n, s, d = I.rmat(10, 16, seed=51)
    full = oracle.count(n, s, d)
    whole = oracle.induced(n, s, d, np.arange(n, dtype=np.int32))
    np.testing.assert_array_equal(whole["T"], full["T"])
    assert whole["avg"] == pytest.approx(full["avg"], rel=1e-14)
    G = nx.Graph()
    G.add_edges_from((int(a), int(b)) for a, b in zip(s, d) if a != b)
    rng = np.random.default_rng(52)
    for k in (1, 5, 50, 300):
        S = rng.choice(n, size=k, replace=False).astype(np.int32)
        r = oracle.induced(n, s, d, S)
        H = nx.Graph()
        H.add_nodes_from(int(x) for x in S)
        H.add_edges_from(G.subgraph([int(x) for x in S]).edges())
        tri = nx.triangles(H)
        np.testing.assert_array_equal(r["T"], np.array([tri[int(x)] for x in S], dtype=np.uint64))
        assert r["avg"] == pytest.approx(nx.average_clustering(H), rel=1e-12)
    with pytest.raises(oracle.OracleError):
        oracle.induced(n, s, d, np.array([1, 2, 1], dtype=np.int32))


def test_sampled_matches_full():
    n, s, d = I.rmat(12, 16, seed=61)
    full = oracle.count(n, s, d, order=1)
    rng = np.random.default_rng(62)
    hubs = np.argsort(full["deg"])[-5:]
    samp = np.unique(np.concatenate([hubs, rng.choice(n, 60, replace=False)])).astype(np.int32)
    r = oracle.sampled(n, s, d, samp)
    np.testing.assert_array_equal(r["T"], full["T"][samp])
    np.testing.assert_array_equal(r["deg"], full["deg"][samp])


def test_rejects_bad_ids():
    with pytest.raises(oracle.OracleError):
        oracle.count(4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(oracle.OracleError):
        oracle.count(4, np.array([0, -1], np.int32), np.array([1, 2], np.int32))


def test_empty_and_degenerate():
    r = oracle.count(0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert r["total"] == 0 and r["avg"] == 0.0 and r["m"] == 0
    r = oracle.count(7, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert r["total"] == 0 and r["avg"] == 0.0 and r["T"].shape == (7,)
    r = oracle.count(3, np.array([0, 1, 2], np.int32), np.array([0, 1, 2], np.int32))
    assert r["m"] == 0 and r["total"] == 0


# ---------------------------------------------------------------------------
# Planted mistakes: each mutant of the oracle's C source must fail a pin.

MUTANTS = {
    "drop_top_vertex_credit": ("          T[w] += 1;\n", "          T[w] += 0;\n"),
    "cc_numerator_not_doubled": ("2.0 * (double)T[v]", "1.0 * (double)T[v]"),
    "keep_self_loops": ("    if (u == v) continue;\n    int64_t a", "    int64_t a"),
    "no_dedup": ("if (i == 0 || key[i] != key[i - 1]) key[m++] = key[i];", "key[m++] = key[i];"),
    "rank_ties_not_broken": ("return da < db || (da == db && a < b);", "return da <= db;"),
    "rank_reversed_id_mode": ("if (order_mode == 0) return a < b;", "if (order_mode == 0) return a > b || a == 0;"),
    "avg_over_nonisolated": ("*avg = g->n > 0 ? sum / (double)g->n : 0.0;",
                             "{ int64_t k = 0; for (int64_t v = 0; v < g->n; ++v) k += g->off[v + 1] > g->off[v];"
                             " *avg = k > 0 ? sum / (double)k : 0.0; }"),
    "mark_wrong_node": ("if (mark[w] != v + 1) continue;", "if (mark[u] != v + 1) continue;"),
}


def _pins_pass(lib_path):
    """A small battery of the pins above, run against a given oracle build."""
    import ctypes
    L = ctypes.CDLL(lib_path)
    P = ctypes.c_void_p
    L.oracle_count.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]

    def run(n, s, d, order):
        s = np.ascontiguousarray(s, np.int32)
        d = np.ascontiguousarray(d, np.int32)
        T = np.zeros(n, np.uint64)
        cc = np.zeros(n)
        deg = np.zeros(n, np.int64)
        tot, avg, m = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_int64()
        rc = L.oracle_count(n, s.size, s.ctypes.data, d.ctypes.data, order, 1, T.ctypes.data, cc.ctypes.data,
                            deg.ctypes.data, ctypes.byref(tot), ctypes.byref(avg), ctypes.byref(m))
        return rc, dict(T=T, cc=cc, total=tot.value, avg=avg.value)

    cases = [F.messy(*F.complete(8), seed=1), (6, np.array([1, 2, 3, 3], np.int32), np.array([2, 3, 1, 4], np.int32))]
    n, s, d = I.rmat(5, 8, seed=9)
    cases.append((n, s, d))
    for n, s, d in cases:
        T, total, cc, avg, _ = brute_force(n, s, d)
        for order in (0, 1):
            rc, r = run(n, s, d, order)
            if rc != 0:
                return False
            try:
                assert_matches(r, T, total, cc, avg)
            except AssertionError:
                return False
    return True


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_planted_mistake_is_caught(mutant, tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    text = open(src).read()
    old, new = MUTANTS[mutant]
    assert old in text, f"mutation anchor for {mutant} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mpath), "-o", str(lib)],
                   check=True)
    assert not _pins_pass(str(lib)), f"mutant {mutant} passed the pins"


def test_unmutated_oracle_passes_battery(tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    lib = tmp_path / "liborig.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", src, "-o", str(lib)], check=True)
    assert _pins_pass(str(lib))


# ---------------------------------------------------------------------------
# edge-existence tests (IsEdge): pinned to the dense adjacency matrix built
# from the raw pairs, to networkx, and to relabelling / noisy-input invariance

def _all_pairs(n, extra=True):
    """Every ordered pair of ids, plus ids just outside [0, n)."""
    qu, qv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    qu, qv = qu.ravel(), qv.ravel()
    if extra:
        bad_u = np.array([-1, n, 0, n + 5, -7, 2**31 - 1], np.int64)
        bad_v = np.array([0, 0, n, 1, -1, 0], np.int64)
        qu, qv = np.concatenate([qu, bad_u]), np.concatenate([qv, bad_v])
    return qu.astype(np.int32), qv.astype(np.int32)


def _edge_expect(n, s, d, qu, qv):
    A = adjacency(n, s, d)
    ok = (qu >= 0) & (qu < n) & (qv >= 0) & (qv < n)
    out = np.full(qu.size, 0xFF, np.uint8)
    out[ok] = A[qu[ok], qv[ok]].astype(np.uint8)
    return out


EDGE_CASES = [
    ("messy_K8", lambda: F.messy(*F.complete(8), seed=3)),
    ("wheel", lambda: F.wheel(17)),
    ("star", lambda: F.star(25)),
    ("rmat6", lambda: I.rmat(6, 8, seed=4)),
    ("er", lambda: (60, *I.er(60, 400, 5))),
    ("loops_only", lambda: (5, np.array([0, 1, 2], np.int32), np.array([0, 1, 2], np.int32))),
    ("no_edges", lambda: (7, np.zeros(0, np.int32), np.zeros(0, np.int32))),
]


@pytest.mark.parametrize("name", [c[0] for c in EDGE_CASES])
def test_has_edges_against_dense_matrix(name):
    n, s, d = dict(EDGE_CASES)[name]()
    qu, qv = _all_pairs(n)
    out = oracle.has_edges(n, s, d, qu, qv)
    np.testing.assert_array_equal(out, _edge_expect(n, s, d, qu, qv))
    # symmetric, never a self pair
    sq = qu.size - 6
    M = out[:sq].reshape(n, n)
    assert np.array_equal(M, M.T) and not M.diagonal().any()


def test_has_edges_against_networkx():
    s, d = I.ba(800, 5, 11)
    G = nx.Graph()
    G.add_nodes_from(range(800))
    G.add_edges_from(zip(s.tolist(), d.tolist()))
    G.remove_edges_from(nx.selfloop_edges(G))
    rng = np.random.default_rng(12)
    qu = rng.integers(0, 800, 20000).astype(np.int32)
    qv = rng.integers(0, 800, 20000).astype(np.int32)
    # half of the queries are input pairs, in either direction
    k = rng.integers(0, s.size, 10000)
    flip = rng.integers(0, 2, 10000).astype(bool)
    qu[:10000] = np.where(flip, d[k], s[k])
    qv[:10000] = np.where(flip, s[k], d[k])
    out = oracle.has_edges(800, s, d, qu, qv)
    ref = np.array([G.has_edge(int(a), int(b)) for a, b in zip(qu, qv)], np.uint8)
    np.testing.assert_array_equal(out, ref)
    assert out[:10000].all()


def test_has_edges_invariant_under_noise_and_relabelling():
    n, s, d = I.rmat(9, 8, seed=21)
    rng = np.random.default_rng(22)
    qu = rng.integers(0, n, 5000).astype(np.int32)
    qv = rng.integers(0, n, 5000).astype(np.int32)
    base = oracle.has_edges(n, s, d, qu, qv)
    n2, s2, d2 = F.messy(n, s, d, seed=23)
    np.testing.assert_array_equal(oracle.has_edges(n2, s2, d2, qu, qv), base)
    n3, s3, d3, perm = F.relabel(n, s, d, seed=24)
    np.testing.assert_array_equal(oracle.has_edges(n3, s3, d3, perm[qu], perm[qv]), base)


EDGE_MUTANTS = {
    "edge_key_not_ordered": ("const uint64_t k = ((uint64_t)(u < v ? u : v) << 32) | (uint64_t)(u < v ? v : u);",
                             "const uint64_t k = ((uint64_t)u << 32) | (uint64_t)v;"),
    "edge_range_off_by_one": ("if (u < 0 || v < 0 || u >= n || v >= n) {\n      out[i] = 0xFF;",
                              "if (u < 0 || v < 0 || u > n || v > n) {\n      out[i] = 0xFF;"),
    "edge_found_inverted": ("sizeof(uint64_t), cmp_u64) != NULL;", "sizeof(uint64_t), cmp_u64) == NULL;"),
}


def _edge_pins_pass(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    P = ctypes.c_void_p
    L.oracle_has_edges.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int64, P, P, P]
    for name, make in EDGE_CASES:
        n, s, d = make()
        s = np.ascontiguousarray(s, np.int32)
        d = np.ascontiguousarray(d, np.int32)
        qu, qv = _all_pairs(n)
        out = np.zeros(qu.size, np.uint8)
        if L.oracle_has_edges(n, s.size, s.ctypes.data, d.ctypes.data, qu.size, qu.ctypes.data, qv.ctypes.data,
                              out.ctypes.data):
            return False
        if not np.array_equal(out, _edge_expect(n, s, d, qu, qv)):
            return False
    return True


@pytest.mark.parametrize("mutant", sorted(EDGE_MUTANTS))
def test_planted_edge_mistake_is_caught(mutant, tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    text = open(src).read()
    old, new = EDGE_MUTANTS[mutant]
    assert old in text, f"mutation anchor for {mutant} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mpath), "-o", str(lib)],
                   check=True)
    assert not _edge_pins_pass(str(lib)), f"mutant {mutant} passed the pins"


def test_unmutated_oracle_passes_edge_battery(tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    lib = tmp_path / "liborig.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", src, "-o", str(lib)], check=True)
    assert _edge_pins_pass(str(lib))


# ---------------------------------------------------------------------------
# core numbers: pinned to naive repeated deletion per k, to networkx, to the
# closed forms of regular families, to invariances and to planted mistakes

def naive_core(n, s, d):
    """core(v) = the largest k such that v survives repeated deletion of the
    nodes of degree < k (the k-core, computed afresh for every k)."""
    A = adjacency(n, s, d).astype(bool)
    core = np.zeros(n, np.int64)
    k = 0
    while True:
        k += 1
        alive = np.ones(n, bool)
        while True:
            deg = (A & alive[None, :]).sum(1) * alive
            drop = alive & (deg < k)
            if not drop.any():
                break
            alive &= ~drop
        if not alive.any():
            return core
        core[alive] = k


CORE_CASES = [
    ("messy_K9", lambda: F.messy(*F.complete(9), seed=5)),
    ("wheel_union", lambda: F.disjoint_union(F.wheel(12), F.windmill(5), F.star(6), F.complete(5))),
    ("rmat7", lambda: I.rmat(7, 8, seed=6)),
    ("er", lambda: (70, *I.er(70, 500, 7))),
    ("ba", lambda: (90, *I.ba(90, 4, 8))),
    ("isolated", lambda: (6, np.array([1, 2], np.int32), np.array([2, 1], np.int32))),
]


@pytest.mark.parametrize("name", [c[0] for c in CORE_CASES])
def test_core_against_naive_deletion(name):
    n, s, d = dict(CORE_CASES)[name]()
    ref = naive_core(n, s, d)
    np.testing.assert_array_equal(oracle.core(n, s, d), ref)
    for k in (0, 1, 2, 3, 5):
        np.testing.assert_array_equal(oracle.core(n, s, d, k_stop=k), np.minimum(ref, k))


def test_core_against_networkx():
    n, s, d = I.rmat(12, 16, seed=9)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(s.tolist(), d.tolist()))
    G.remove_edges_from(nx.selfloop_edges(G))
    ref = nx.core_number(G)
    np.testing.assert_array_equal(oracle.core(n, s, d), np.array([ref[v] for v in range(n)]))


@pytest.mark.parametrize("case,expect", [
    ("complete", lambda: (F.complete(11), 10)),
    ("ring", lambda: (F.ring(30), 2)),
    ("path", lambda: (F.path(20), 1)),
    ("star", lambda: (F.star(15), 1)),
    ("tree", lambda: (F.random_tree(40, 3), 1)),
    ("grid", lambda: (F.grid(5, 7), 2)),
    ("bipartite", lambda: (F.complete_bipartite(4, 9), 4)),
    ("wheel", lambda: (F.wheel(10), 3)),
    ("windmill", lambda: (F.windmill(6), 2)),
    ("lattice", lambda: (F.ring_lattice(40, 6), 6)),
])
def test_core_closed_forms(case, expect):
    (n, s, d), k = expect()
    assert np.all(oracle.core(n, s, d) == k)


def test_core_invariant_under_noise_and_relabelling():
    n, s, d = I.rmat(10, 8, seed=10)
    base = oracle.core(n, s, d)
    n2, s2, d2 = F.messy(n, s, d, seed=11)
    np.testing.assert_array_equal(oracle.core(n2, s2, d2), base)
    n3, s3, d3, perm = F.relabel(n, s, d, seed=12)
    got = oracle.core(n3, s3, d3)
    np.testing.assert_array_equal(got[perm], base)


CORE_MUTANTS = {
    "core_ties_lowered": ("      if (d[u] > d[v]) {", "      if (d[u] >= d[v]) {"),
    "core_bucket_not_moved": ("        bin[du]++;\n        d[u]--;", "        d[u]--;"),
    "core_stop_ignored": ("core[v] = (int32_t)(k_stop >= 0 && d[v] > k_stop ? k_stop : d[v]);",
                          "core[v] = (int32_t)d[v];"),
}


def _core_pins_pass(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    P = ctypes.c_void_p
    L.oracle_core.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int32, P]
    for name, make in CORE_CASES:
        n, s, d = make()
        s = np.ascontiguousarray(s, np.int32)
        d = np.ascontiguousarray(d, np.int32)
        ref = naive_core(n, s, d)
        for k in (-1, 2):
            out = np.zeros(n, np.int32)
            if L.oracle_core(n, s.size, s.ctypes.data, d.ctypes.data, k, out.ctypes.data):
                return False
            if not np.array_equal(out, ref if k < 0 else np.minimum(ref, k)):
                return False
    return True


@pytest.mark.parametrize("mutant", sorted(CORE_MUTANTS))
def test_planted_core_mistake_is_caught(mutant, tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    text = open(src).read()
    old, new = CORE_MUTANTS[mutant]
    assert old in text, f"mutation anchor for {mutant} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mpath), "-o", str(lib)],
                   check=True)
    assert not _core_pins_pass(str(lib)), f"mutant {mutant} passed the pins"


def test_unmutated_oracle_passes_core_battery(tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    lib = tmp_path / "liborig.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", src, "-o", str(lib)], check=True)
    assert _core_pins_pass(str(lib))


# ---------------------------------------------------------------------------
# 4-clique counts: pinned to brute force over all 4-subsets, to networkx's
# clique enumeration, to closed forms, invariances and planted mistakes

def brute_k4(n, s, d):
    A = adjacency(n, s, d).astype(bool)
    return sum(1 for q in itertools.combinations(range(n), 4)
               if all(A[a, b] for a, b in itertools.combinations(q, 2)))


K4_CASES = [
    ("messy_K9", lambda: F.messy(*F.complete(9), seed=5)),
    ("rmat5", lambda: I.rmat(5, 8, seed=6)),
    ("er", lambda: (24, *I.er(24, 150, 7))),
    ("ba", lambda: (26, *I.ba(26, 5, 8))),
    ("union", lambda: F.disjoint_union(F.complete(6), F.wheel(3), F.ring_lattice(12, 6), F.windmill(3))),
]


@pytest.mark.parametrize("name", [c[0] for c in K4_CASES])
def test_k4_against_brute_force(name):
    n, s, d = dict(K4_CASES)[name]()
    ref = brute_k4(n, s, d)
    assert oracle.k4(n, s, d, order=0) == ref
    assert oracle.k4(n, s, d, order=1) == ref


def test_k4_against_networkx():
    for n, s, d in (I.rmat(9, 8, seed=13), (2000, *I.ba(2000, 5, 14))):
        G = nx.Graph()
        G.add_edges_from(zip(s.tolist(), d.tolist()))
        G.remove_edges_from(nx.selfloop_edges(G))
        ref = sum(1 for c in nx.enumerate_all_cliques(G) if len(c) == 4)
        assert oracle.k4(n, s, d) == ref


@pytest.mark.parametrize("case,expect", [
    ("complete", lambda: (F.complete(13), 715)),
    ("k4_wheel", lambda: (F.wheel(3), 1)),
    ("wheel", lambda: (F.wheel(9), 0)),
    ("bipartite", lambda: (F.complete_bipartite(5, 6), 0)),
    ("windmill", lambda: (F.windmill(7), 0)),
    ("lattice4", lambda: (F.ring_lattice(40, 4), 0)),
    ("lattice6", lambda: (F.ring_lattice(40, 6), 40)),
])
def test_k4_closed_forms(case, expect):
    (n, s, d), k = expect()
    assert oracle.k4(n, s, d) == k


def test_k4_invariant_under_noise_and_relabelling():
    n, s, d = I.rmat(9, 8, seed=15)
    base = oracle.k4(n, s, d)
    assert oracle.k4(*F.messy(n, s, d, seed=16)) == base
    n3, s3, d3, _ = F.relabel(n, s, d, seed=17)
    assert oracle.k4(n3, s3, d3) == base


K4_MUTANTS = {
    "k4_no_rank_on_x": ("if (og_below(&g, order_mode, w, x) && m1[x] == u + 1) m2[x] = stamp;",
                        "if (m1[x] == u + 1) m2[x] = stamp;"),
    "k4_last_mark_wrong": ("if (og_below(&g, order_mode, x, z) && m2[z] == stamp) count += 1;",
                           "if (og_below(&g, order_mode, x, z) && m1[z] == u + 1) count += 1;"),
    "k4_stamp_not_advanced": ("          ++stamp;\n", "\n"),
}


def _k4_pins_pass(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    P = ctypes.c_void_p
    L.oracle_k4.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int, P]
    for name, make in K4_CASES:
        n, s, d = make()
        s = np.ascontiguousarray(s, np.int32)
        d = np.ascontiguousarray(d, np.int32)
        ref = brute_k4(n, s, d)
        for order in (0, 1):
            tot = ctypes.c_uint64()
            if L.oracle_k4(n, s.size, s.ctypes.data, d.ctypes.data, order, 1, ctypes.byref(tot)):
                return False
            if tot.value != ref:
                return False
    return True


@pytest.mark.parametrize("mutant", sorted(K4_MUTANTS))
def test_planted_k4_mistake_is_caught(mutant, tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    text = open(src).read()
    old, new = K4_MUTANTS[mutant]
    assert old in text, f"mutation anchor for {mutant} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mpath), "-o", str(lib)],
                   check=True)
    assert not _k4_pins_pass(str(lib)), f"mutant {mutant} passed the pins"


def test_unmutated_oracle_passes_k4_battery(tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    lib = tmp_path / "liborig.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", src, "-o", str(lib)], check=True)
    assert _k4_pins_pass(str(lib))


# ---------------------------------------------------------------------------
# R-MAT edges (the device generator's definition): pinned to SplitMix64's
# published test vector, to the host input generator (independent code),
# to the one-quadrant closed forms, to the quadrant frequencies, and by
# planted mistakes

def test_splitmix64_published_vector():
    g = json.load(open(os.path.join(HERE, "golden", "splitmix64.json")))
    out = oracle.splitmix64(g["state"], len(g["outputs"]))
    assert [int(x) for x in out] == [int(x) for x in g["outputs"]]


RMAT_MATCH = [(1, 0, 0.1), (4, 3, 0.0), (9, 7, 0.1), (11, 2**64 - 1, 0.5), (12, 12, 1.0)]


@pytest.mark.parametrize("scale,seed,noise", RMAT_MATCH)
def test_rmat_equals_input_generator(scale, seed, noise):
    n, s, d = I.rmat(scale, 8, seed=seed, noise=noise, permute=False)
    s2, d2 = oracle.rmat(scale, 8 << scale, seed=seed, noise=noise)
    assert np.array_equal(s, s2) and np.array_equal(d, d2)
    _, s3, d3 = I.rmat(scale, 8, seed=seed, noise=noise, permute=True)
    s4, d4 = oracle.rmat(scale, 8 << scale, seed=seed, noise=noise, perm=I.rmat_perm(scale, seed))
    assert np.array_equal(s3, s4) and np.array_equal(d3, d4)


@pytest.mark.parametrize("q,corner", [(0, (0, 0)), (1, (0, 1)), (2, (1, 0)), (3, (1, 1))])
@pytest.mark.parametrize("noise", [0.0, 0.5])
def test_rmat_one_quadrant_closed_forms(q, corner, noise):
    # all weight on one quadrant: every level picks it, so every edge is
    # the corner (0 or n-1, 0 or n-1)
    scale = 7
    abcd = [0.0] * 4
    abcd[q] = 1.0
    s, d = oracle.rmat(scale, 3000, abcd=abcd, noise=noise, seed=5)
    n = 1 << scale
    assert (s == corner[0] * (n - 1)).all() and (d == corner[1] * (n - 1)).all()


def test_rmat_quadrant_frequencies():
    # noise 0: at every level the quadrant is (a, b, c, d)-distributed,
    # independently; checked per level within 5 sigma
    scale, m = 6, 200_000
    for abcd in ((0.25, 0.25, 0.25, 0.25), (0.57, 0.19, 0.19, 0.05)):
        s, d = oracle.rmat(scale, m, abcd=abcd, noise=0.0, seed=11)
        for lvl in range(scale):
            bit = scale - 1 - lvl
            q = ((s >> bit) & 1) * 2 + ((d >> bit) & 1)
            freq = np.bincount(q, minlength=4) / m
            for k in range(4):
                sigma = (abcd[k] * (1 - abcd[k]) / m) ** 0.5
                assert abs(freq[k] - abcd[k]) < 5 * sigma + 1e-12, (abcd, lvl, k, freq)


def test_rmat_indexed_edges_equal_full_run():
    s, d = oracle.rmat(10, 5000, seed=21)
    idx = np.array([0, 1, 17, 2047, 4999, 3333, 17], np.int64)
    s2, d2 = oracle.rmat(10, idx=idx, seed=21)
    assert np.array_equal(s[idx], s2) and np.array_equal(d[idx], d2)


RMAT_MUTANTS = {
    "rmat_bits_swapped": ("u = (u << 1) | (uint32_t)(q >> 1);", "u = (u << 1) | (uint32_t)(q & 1);"),
    "rmat_noise_sign": ("(1.0 + noise * (2.0 * h / 65535.0 - 1.0))", "(1.0 + noise * (1.0 - 2.0 * h / 65535.0))"),
    "rmat_draw_offset": ("sm_out(S + sm_gamma * (kk + 2u))", "sm_out(S + sm_gamma * (kk + 3u))"),
    "rmat_sum_drops_last": ("(((p[0] + p[1]) + p[2]) + p[3])", "((p[0] + p[1]) + p[2])"),
}


def _rmat_pins_pass(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    P, dbl = ctypes.c_void_p, ctypes.c_double
    L.oracle_rmat.argtypes = [ctypes.c_int, dbl, dbl, dbl, dbl, dbl, ctypes.c_uint64, ctypes.c_int64, P, P, P, P]

    def run(scale, m, abcd, noise, seed):
        s = np.zeros(m, np.int32)
        d = np.zeros(m, np.int32)
        if L.oracle_rmat(scale, *abcd, noise, seed, m, None, None, s.ctypes.data, d.ctypes.data):
            return None
        return s, d

    for scale, seed, noise in RMAT_MATCH[:3]:
        _, s, d = I.rmat(scale, 8, seed=seed, noise=noise, permute=False)
        r = run(scale, 8 << scale, (0.57, 0.19, 0.19, 0.05), noise, seed)
        if r is None or not (np.array_equal(r[0], s) and np.array_equal(r[1], d)):
            return False
    for q, corner in ((1, (0, 1)), (2, (1, 0))):
        abcd = [0.0] * 4
        abcd[q] = 1.0
        r = run(5, 500, abcd, 0.0, 3)
        if r is None or not ((r[0] == corner[0] * 31).all() and (r[1] == corner[1] * 31).all()):
            return False
    return True


@pytest.mark.parametrize("mutant", sorted(RMAT_MUTANTS))
def test_planted_rmat_mistake_is_caught(mutant, tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    text = open(src).read()
    old, new = RMAT_MUTANTS[mutant]
    assert old in text, f"mutation anchor for {mutant} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mpath), "-o", str(lib)],
                   check=True)
    assert not _rmat_pins_pass(str(lib)), f"mutant {mutant} passed the pins"


def test_unmutated_oracle_passes_rmat_battery(tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    lib = tmp_path / "liborig.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", src, "-o", str(lib)], check=True)
    assert _rmat_pins_pass(str(lib))


def test_count_timed_sample_partitions_the_triangles():
    """The node-sampled timing entry finds exactly the triangles whose
    lowest-ranked vertex is sampled: over all offsets of one stride the
    samples add up to the whole count (both rank orders), and stride 1 is the
    whole count."""
    from paper_1606_07550_amd import inputs as I
    n, s, d = I.rmat(12, 16, seed=81)
    for order in (0, 1):
        full = oracle.count(n, s, d, order=order)["total"]
        assert oracle.count_timed(n, s, d, order=order, stride=1)["tri"] == full
        parts = [oracle.count_timed(n, s, d, order=order, stride=7, offset=o, stride1=7) for o in range(7)]
        assert sum(p["tri"] for p in parts) == full and all(p["tri"] < full for p in parts)
        assert all(p["tri1"] == p["tri"] for p in parts)  # one thread finds the same
    with pytest.raises(oracle.OracleError):
        oracle.count_timed(n, s, d, stride=4, offset=4)


# ---------------------------------------------------------------------------
# G(n, m) and Barabasi-Albert generators of the oracle (the paper's table of
# graph generators, Section 4). Pins: the defining properties of each model
# (exactly m distinct loop-free pairs; a uniform m-subset, by frequencies and
# a chi-square over all subsets of a tiny pair set; the complete graph at
# m = N; the prefix property of first-m-distinct draws; k distinct earlier
# targets per BA node, the seed clique, attachment in proportion to degree,
# the heavy degree tail), and planted mistakes that each fail one of them.

def _er_pins_pass(er):
    from itertools import combinations
    for n, m, seed in ((2, 1, 1), (7, 21, 2), (9, 36, 3), (50, 300, 4), (2000, 20000, 5), (100, 0, 6)):
        s, d = er(n, m, seed)
        if s is None or s.size != m:
            return False
        if m == 0:
            continue
        if s.min() < 0 or d.min() < 0 or s.max() >= n or d.max() >= n or np.any(s == d):
            return False
        key = np.minimum(s, d).astype(np.int64) * n + np.maximum(s, d)
        if np.unique(key).size != m:
            return False
        if m == n * (n - 1) // 2 and np.unique(key).size != m:  # complete graph
            return False
    # prefix property: G(n, m') is the first m' edges of G(n, m)
    s1, d1 = er(300, 2000, 7)
    s2, d2 = er(300, 700, 7)
    if s1 is None or s2 is None or not (np.array_equal(s1[:700], s2) and np.array_equal(d1[:700], d2)):
        return False
    # uniform m-subsets: n = 5 (N = 10), m = 3 over 12,000 seeds
    pairs = list(combinations(range(5), 2))
    subsets = {frozenset(c): i for i, c in enumerate(combinations(range(10), 3))}
    cnt = np.zeros(len(subsets))
    pair_cnt = np.zeros(10)
    flips = 0
    R = 12000
    for seed in range(R):
        s, d = er(5, 3, 1000 + seed)
        ids = [pairs.index((min(a, b), max(a, b))) for a, b in zip(s.tolist(), d.tolist())]
        cnt[subsets[frozenset(ids)]] += 1
        pair_cnt[ids] += 1
        flips += int(np.sum(s > d))
    exp = R / len(subsets)
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    if chi2 > 200.0:  # 119 degrees of freedom: p below 1e-5
        return False
    p = 3 / 10
    if np.any(np.abs(pair_cnt - R * p) > 5 * np.sqrt(R * p * (1 - p))):
        return False
    if abs(flips - 1.5 * R) > 5 * np.sqrt(3 * R * 0.25):
        return False
    return True


def _ba_pins_pass(ba):
    for n, k, seed in ((3, 2, 1), (40, 1, 2), (300, 3, 3), (2000, 5, 4), (500, 16, 5)):
        s, d = ba(n, k, seed)
        if s is None:
            return False
        m = k * (k + 1) // 2 + (n - k - 1) * k
        if s.size != m:
            return False
        es = k * (k + 1) // 2
        seed_pairs = sorted(zip(s[:es].tolist(), d[:es].tolist()))
        if seed_pairs != [(i, j) for i in range(k + 1) for j in range(i + 1, k + 1)]:
            return False
        sv = s[es:].reshape(-1, k)
        dv = d[es:].reshape(-1, k)
        v = np.arange(k + 1, n)
        if not np.all(sv == v[:, None]) or not np.all(dv < v[:, None]) or not np.all(dv >= 0):
            return False
        if any(len(set(row)) != k for row in dv.tolist()):
            return False
    # attachment in proportion to degree: the first target of node v = 20
    # (k = 2) against the degrees of the graph before v, over many seeds
    k, v = 2, 20
    es = k * (k + 1) // 2
    ev = es + (v - k - 1) * k
    obs = np.zeros(v)
    expct = np.zeros(v)
    var = 0.0
    for seed in range(3000):
        s, d = ba(v + 1, k, 500 + seed)
        deg = np.bincount(np.concatenate([s[:ev], d[:ev]]), minlength=v).astype(np.float64)
        prob = deg / (2.0 * ev)
        obs[d[ev]] += 1
        expct += prob
        var += float((prob * (1 - prob)).sum())
    if np.any(np.abs(obs - expct) > 5 * np.sqrt(np.maximum(expct, 1.0))):
        return False
    # a heavy tail: uniform attachment would keep the largest degree near
    # k ln n (about 46 here); preferential attachment grows it like sqrt(n)
    s, d = ba(100000, 4, 9)
    if np.bincount(np.concatenate([s, d])).max() < 300:
        return False
    return True


def _lib_gens(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    P = ctypes.c_void_p
    L.oracle_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, P, P]
    L.oracle_ba.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, P, P]

    def er(n, m, seed):
        s = np.zeros(m, np.int32)
        d = np.zeros(m, np.int32)
        return (s, d) if L.oracle_er(n, m, seed, s.ctypes.data, d.ctypes.data) == 0 else (None, None)

    def ba(n, k, seed):
        m = k * (k + 1) // 2 + (n - k - 1) * k
        s = np.zeros(m, np.int32)
        d = np.zeros(m, np.int32)
        return (s, d) if L.oracle_ba(n, k, seed, s.ctypes.data, d.ctypes.data) == 0 else (None, None)
    return er, ba


def test_er_oracle_pins():
    assert _er_pins_pass(oracle.er)


def test_ba_oracle_pins():
    assert _ba_pins_pass(oracle.ba)


GEN_MUTANTS = {
    "er_no_dedup": ("    if (seen) continue;\n    set[h] = x + 1;", "    set[h] = x + 1;"),
    "er_row_off_by_one": ("if ((uint64_t)(mid * n - mid * (mid + 1) / 2) <= t) lo = mid;",
                          "if ((uint64_t)(mid * n - mid * (mid + 1) / 2) < t) lo = mid;"),
    "er_low_pairs_only": ("const uint64_t x = mul_hi(w, N);", "const uint64_t x = mul_hi(w, N) / 2;"),
    "er_no_flip": ("src[got] = (int32_t)((w & 1u) ? j : i);", "src[got] = (int32_t)i;"),
    "ba_sources_only": ("c = (r & 1u) ? dst[r >> 1] : src[r >> 1];", "c = src[r >> 1];"),
    "ba_span_own_edges": ("2u * (uint64_t)ev);", "2u * (uint64_t)ev + 2u);"),
    "ba_not_distinct": ("for (int32_t q = 0; q < j; ++q) dup |= dst[ev + q] == c;\n        if (!dup) break;",
                        "if (!dup) break;"),
}


@pytest.mark.parametrize("mutant", sorted(GEN_MUTANTS))
def test_planted_generator_mistake_is_caught(mutant, tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    text = open(src).read()
    old, new = GEN_MUTANTS[mutant]
    assert old in text, f"mutation anchor for {mutant} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mpath), "-o", str(lib)],
                   check=True)
    er, ba = _lib_gens(str(lib))
    if mutant.startswith("er"):
        assert not _er_pins_pass(er), f"mutant {mutant} passed the pins"
    else:
        assert not _ba_pins_pass(ba), f"mutant {mutant} passed the pins"


# ---------------------------------------------------------------------------
# 5-clique counts: pinned to brute force over all 5-subsets, to networkx's
# clique enumeration, to closed forms (C(n, 5) for K_n; n for the ring
# lattice with 4 neighbours on each side, whose 5-cliques are its windows of
# 5 consecutive nodes; 0 where no 5 nodes are pairwise adjacent), invariances
# and planted mistakes

def brute_k5(n, s, d):
    A = adjacency(n, s, d).astype(bool)
    nb = [set(np.flatnonzero(A[v]).tolist()) for v in range(n)]
    cnt = 0
    for q in itertools.combinations(range(n), 3):  # extend triangles: fewer subsets to visit
        a, b, c = q
        if b in nb[a] and c in nb[a] and c in nb[b]:
            common = [z for z in nb[a] & nb[b] & nb[c] if z > c]
            cnt += sum(1 for i, y in enumerate(common) for z in common[i + 1:] if z in nb[y])
    return cnt


K5_CASES = [
    ("messy_K10", lambda: F.messy(*F.complete(10), seed=25)),
    ("rmat6", lambda: I.rmat(6, 12, seed=26)),
    ("er", lambda: (26, *I.er(26, 220, 27))),
    ("ba", lambda: (30, *I.ba(30, 7, 28))),
    ("union", lambda: F.disjoint_union(F.complete(7), F.wheel(4), F.ring_lattice(14, 8), F.windmill(3))),
]


@pytest.mark.parametrize("name", [c[0] for c in K5_CASES])
def test_k5_against_brute_force(name):
    n, s, d = dict(K5_CASES)[name]()
    ref = brute_k5(n, s, d)
    assert ref > 0 or name == "ba"
    assert oracle.k5(n, s, d, order=0) == ref
    assert oracle.k5(n, s, d, order=1) == ref


def test_brute_k5_itself_on_closed_forms():
    from math import comb
    for k in (5, 6, 9):
        assert brute_k5(*F.complete(k)) == comb(k, 5)
    assert brute_k5(*F.ring_lattice(14, 8)) == 14 and brute_k5(*F.wheel(6)) == 0


def test_k5_against_networkx():
    for n, s, d in (I.rmat(9, 10, seed=33), (2000, *I.ba(2000, 6, 34))):
        G = nx.Graph()
        G.add_edges_from(zip(s.tolist(), d.tolist()))
        G.remove_edges_from(nx.selfloop_edges(G))
        ref = sum(1 for c in nx.enumerate_all_cliques(G) if len(c) == 5)
        assert oracle.k5(n, s, d) == ref


@pytest.mark.parametrize("case,expect", [
    ("complete", lambda: (F.complete(13), 1287)),
    ("k5", lambda: (F.complete(5), 1)),
    ("wheel", lambda: (F.wheel(9), 0)),
    ("bipartite", lambda: (F.complete_bipartite(6, 6), 0)),
    ("lattice6", lambda: (F.ring_lattice(40, 6), 0)),
    ("lattice8", lambda: (F.ring_lattice(40, 8), 40)),
])
def test_k5_closed_forms(case, expect):
    (n, s, d), k = expect()
    assert oracle.k5(n, s, d) == k


def test_k5_invariant_under_noise_and_relabelling():
    n, s, d = I.rmat(9, 12, seed=35)
    base = oracle.k5(n, s, d)
    assert base > 0
    assert oracle.k5(*F.messy(n, s, d, seed=36)) == base
    n3, s3, d3, _ = F.relabel(n, s, d, seed=37)
    assert oracle.k5(n3, s3, d3) == base


K5_MUTANTS = {
    "k5_no_rank_on_y": ("if (og_below(&g, order_mode, x, y) && m2[y] == s2) m3[y] = s3;",
                        "if (m2[y] == s2) m3[y] = s3;"),
    "k5_last_mark_wrong": ("if (og_below(&g, order_mode, y, z) && m3[z] == s3) count += 1;",
                           "if (og_below(&g, order_mode, y, z) && m2[z] == s2) count += 1;"),
    "k5_inner_stamp_not_advanced": ("            ++s3;\n", "\n"),
}


def _k5_pins_pass(lib_path):
    import ctypes
    L = ctypes.CDLL(lib_path)
    P = ctypes.c_void_p
    L.oracle_k5.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int, P]
    for name, make in K5_CASES:
        n, s, d = make()
        s = np.ascontiguousarray(s, np.int32)
        d = np.ascontiguousarray(d, np.int32)
        ref = brute_k5(n, s, d)
        for order in (0, 1):
            tot = ctypes.c_uint64()
            if L.oracle_k5(n, s.size, s.ctypes.data, d.ctypes.data, order, 1, ctypes.byref(tot)):
                return False
            if tot.value != ref:
                return False
    return True


@pytest.mark.parametrize("mutant", sorted(K5_MUTANTS))
def test_planted_k5_mistake_is_caught(mutant, tmp_path):
    src = os.path.join(os.path.dirname(HERE), "oracle", "tricc_oracle.c")
    text = open(src).read()
    old, new = K5_MUTANTS[mutant]
    assert old in text, f"mutation anchor for {mutant} not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(text.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11", str(mpath), "-o", str(lib)],
                   check=True)
    assert not _k5_pins_pass(str(lib)), f"mutant {mutant} passed the pins"

"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Counts are compared bit for bit; FP32 clustering coefficients within 1e-6
relative of the FP64 oracle with exact zeros; the FP64 average within 1e-6
relative (it is summed in FP64, so it is in fact much closer).
"""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1606_07550_amd as P
from paper_1606_07550_amd import _native as N
from paper_1606_07550_amd import inputs as I
from paper_1606_07550_amd.inputs import fixtures as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CC_RTOL = 1e-6


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def gpu_count(n, s, d, tuning=None):
    print(f"[gpu_count] n={n} m_raw={len(s)} tuning={tuning}", flush=True)
    g = P.Graph(n, to_dev(s), to_dev(d), tuning=tuning)
    out = g.count()
    torch.cuda.synchronize()
    r = {
        "T": out["T"].cpu().numpy().view(np.uint64),
        "cc": out["cc"].cpu().numpy(),
        "total": int(out["total"].cpu().numpy().view(np.uint64)[0]),
        "avg": float(out["avg"].cpu().item()),
        "info": g.info,
        "graph": g,
        "check": g.count_check(),
    }
    return r


def check_against(r, ref, n):
    np.testing.assert_array_equal(r["T"], ref["T"])
    assert r["total"] == ref["total"]
    # the total comes from the intersection kernels' own counters, not from T
    assert r["check"] == (r["total"], int(r["T"].sum(dtype=np.uint64)))
    assert int(r["T"].sum(dtype=np.uint64)) == 3 * r["total"]
    cc_ref = ref["cc"]
    np.testing.assert_allclose(r["cc"].astype(np.float64), cc_ref, rtol=CC_RTOL, atol=0)
    assert np.array_equal(r["cc"] == 0, cc_ref == 0)
    if n:
        assert abs(r["avg"] - ref["avg"]) <= CC_RTOL * abs(ref["avg"])
    else:
        assert r["avg"] == 0.0
    assert r["info"]["m"] == ref["m"]


def parity(n, s, d, tuning=None, order=1):
    ref = oracle.count(n, s, d, order=order)
    r = gpu_count(n, s, d, tuning)
    check_against(r, ref, n)
    return r, ref


FIXTURES = {
    "K1": F.complete(1), "K2": F.complete(2), "K3": F.complete(3), "K7": F.complete(7), "K40": F.complete(40),
    "ring3": F.ring(3), "ring50": F.ring(50), "star100": F.star(100), "path30": F.path(30),
    "tree500": F.random_tree(500, 3), "grid": F.grid(20, 31), "Kab": F.complete_bipartite(9, 13),
    "bip": F.random_bipartite(80, 70, 0.2, 4), "wheel33": F.wheel(33), "windmill12": F.windmill(12),
    "lattice": F.ring_lattice(301, 10),
    "union": F.disjoint_union(F.complete(9), F.wheel(7), F.ring(10), F.windmill(4)),
}


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_fixture_families(name):
    parity(*FIXTURES[name])


def test_golden_small_graphs():
    import json
    import os
    from fractions import Fraction
    with open(os.path.join(os.path.dirname(__file__), "golden", "small_graphs.json")) as f:
        data = json.load(f)
    for g in data["graphs"]:
        e = np.array(g["edges"], dtype=np.int32).reshape(-1, 2)
        r = gpu_count(g["n"], e[:, 0], e[:, 1])
        assert r["total"] == g["total"]
        np.testing.assert_array_equal(r["T"], np.array(g["T"], dtype=np.uint64))
        np.testing.assert_allclose(r["cc"], [float(Fraction(c)) for c in g["cc"]], rtol=CC_RTOL)
        assert r["avg"] == pytest.approx(float(Fraction(g["avg"])), rel=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_er_config(seed):
    """G(n=10^4, m=10^5): the small configuration."""
    s, d = I.er(10_000, 100_000, seed)
    parity(10_000, s, d)


@pytest.mark.parametrize("scale", [6, 9, 12, 14, 16])
def test_rmat_small_scales(scale):
    n, s, d = I.rmat(scale, 16, seed=100 + scale)
    parity(n, s, d)


@pytest.mark.parametrize("n,k", [(200, 2), (5000, 7), (30000, 16)])
def test_ba(n, k):
    s, d = I.ba(n, k, n + k)
    parity(n, s, d)


def test_edge_cases():
    e = np.zeros(0, np.int32)
    for n in (0, 1, 5):
        r = gpu_count(n, e, e)
        assert r["total"] == 0 and r["avg"] == 0.0 and r["T"].size == n and not np.any(r["T"])
    loops = np.arange(6, dtype=np.int32)
    r = gpu_count(6, loops, loops)
    assert r["info"]["m"] == 0 and r["total"] == 0
    parity(2, np.array([0], np.int32), np.array([1], np.int32))
    parity(3, np.array([0, 1, 2, 0, 0], np.int32), np.array([1, 2, 0, 1, 1], np.int32))


def test_out_of_range_ids_are_rejected():
    for bad in ([0, 5], [0, -1], [2**31 - 1, 0]):
        with pytest.raises(N.TriccError) as ei:
            P.Graph(5, to_dev(np.array(bad, np.int32)), to_dev(np.array([1, 2], np.int32)))
        assert ei.value.status == N.TRICC_ERANGE


def test_input_order_and_noise_invariance():
    n, s, d = I.rmat(13, 16, seed=7)
    r0, _ = parity(n, s, d)
    r1 = gpu_count(*F.messy(n, s, d, seed=8))
    np.testing.assert_array_equal(r1["T"], r0["T"])
    np.testing.assert_array_equal(r1["cc"], r0["cc"])
    assert r1["avg"] == r0["avg"]
    n2, s2, d2, perm = F.relabel(n, s, d, seed=9)
    r2 = gpu_count(n2, s2, d2)
    np.testing.assert_array_equal(r2["T"][perm], r0["T"])


def test_repeatable_bit_identical():
    n, s, d = I.rmat(14, 16, seed=11)
    g = P.Graph(n, to_dev(s), to_dev(d))
    outs = []
    for _ in range(3):
        o = g.count()
        torch.cuda.synchronize()
        outs.append({k: v.clone().cpu() for k, v in o.items()})
    for o in outs[1:]:
        for k in o:
            assert torch.equal(o[k], outs[0][k]), k


def test_csr_and_dag_structure():
    n, s, d = I.rmat(12, 16, seed=13)
    ref = oracle.count(n, s, d, order=1)
    g = P.Graph(n, to_dev(s), to_dev(d))
    A = {k: v.cpu().numpy() for k, v in g.arrays().items()}
    off, deg, adj = A["off"], A["deg"], A["adj"]
    np.testing.assert_array_equal(deg, ref["deg"])
    rows = [adj[off[v]:off[v] + deg[v]] for v in range(n)]
    for v in range(n):
        r = rows[v]
        assert np.all(np.diff(r) > 0)  # sorted, unique
        assert not np.any(r == v)
    # symmetric
    pairs = {(v, int(w)) for v in range(n) for w in rows[v]}
    assert all((w, v) in pairs for (v, w) in pairs)
    doff, dcol = A["doff"], A["dcol"]
    m = ref["m"]
    assert doff[-1] == m
    dplus = np.diff(doff)
    assert dplus.max() <= math.sqrt(2 * m)
    for v in range(n):
        out = dcol[doff[v]:doff[v + 1]]
        assert np.all(np.diff(out) > 0)
        assert all((deg[v], v) < (deg[w], w) for w in out.tolist())
    # algorithmic sizes: sum over DAG edges u->w of d+(u) + d+(w)
    info = g.stats()
    src_of = np.repeat(np.arange(n), dplus)
    assert info["list_elems"] == int((dplus[src_of] + dplus[dcol]).sum())
    assert sum(info["bin_edges"]) == int(dplus[dplus >= 2].sum())


def _tuning_all_to(variant, limit_bins=None):
    t = P.default_tuning()
    for b in range(N.NUM_BINS - 1):
        t.bin_limit[b] = 0
    for b in range(N.NUM_BINS):
        t.bin_variant[b] = variant
    t.min_side = 0
    return t


MIN_SIDE_TUNINGS = [
    {"bin_limit": [16, 64, 256, 1024, 4096], "bin_variant": [0, 1, 2, 3, 4, 8], "min_side": 1},
    {"bin_limit": [4, 8, 32, 128, 512], "bin_variant": [0, 1, 2, 3, 4, 8], "min_side": 1},
    {"bin_limit": [16, 16, 16, 16, 64], "bin_variant": [0, 0, 0, 0, 1, 8], "min_side": 1},
    {"bin_limit": [16, 64, 256, 1024, 4096], "bin_variant": [0, 1, 2, 3, 4, 8], "min_side": 0},
    {"bin_limit": [32, 64, 256, 1024, 2048], "bin_variant": [1, 1, 7, 5, 6, 8], "min_side": 1},
    # cuckoo tables
    {"bin_limit": [16, 64, 256, 1024, 4096], "bin_variant": [10, 11, 12, 13, 14, 9], "min_side": 1},
    {"bin_limit": [64, 256, 512, 1024, 2048], "bin_variant": [11, 17, 15, 13, 16, 8], "min_side": 1},
    {"bin_limit": [4, 8, 32, 128, 512], "bin_variant": [10, 10, 11, 12, 13, 8], "min_side": 1},
    # four short-list nodes per wavefront, the longer ones of the bin one by one
    {"bin_limit": [64, 256, 640, 1024, 4096], "bin_variant": [21, 19, 15, 20, 20, 9], "min_side": 1},
    {"bin_limit": [64, 256, 640, 1024, 4096], "bin_variant": [22, 19, 15, 20, 20, 9], "min_side": 1},
    {"bin_limit": [8, 24, 64, 256, 1024], "bin_variant": [21, 22, 21, 12, 13, 8], "min_side": 1},
    # half-full tables
    {"bin_limit": [64, 256, 512, 1024, 4096], "bin_variant": [21, 23, 24, 26, 20, 9], "min_side": 1},
    {"bin_limit": [32, 128, 512, 1024, 2048], "bin_variant": [22, 23, 25, 26, 20, 8], "min_side": 1},
]


@pytest.mark.parametrize("ti", range(len(MIN_SIDE_TUNINGS)))
def test_min_side_split(ti):
    """Edges counted from the shorter out-list (in-list side for w) under
    several limit sets; in-lists longer than one chunk occur in R-MAT."""
    tun = MIN_SIDE_TUNINGS[ti]
    cases = [I.rmat(14, 16, seed=41), I.rmat(16, 16, seed=42), F.complete(300),
             F.disjoint_union(F.complete(40), F.wheel(30), F.windmill(7))]
    s, d = I.ba(20000, 9, 43)
    cases.append((20000, s, d))
    for n, s, d in cases:
        ref = oracle.count(n, s, d, order=1)
        g = P.Graph(n, to_dev(s), to_dev(d))
        mo = g.info["max_outdeg"]
        if P.variant_capacity(tun["bin_variant"][5]) < mo:
            continue
        g.retune(tun)
        if tun["min_side"] and n > 1000:
            assert sum(g.info["bin_in_items"]) > 0
        o = g.count()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o["T"].cpu().numpy().view(np.uint64), ref["T"])
        assert int(o["total"].cpu().numpy().view(np.uint64)[0]) == ref["total"]
        info = g.stats()
        dplus = np.diff(g.arrays()["doff"].cpu().numpy())
        assert sum(info["bin_edges"]) == int(dplus[dplus >= 2].sum())


@pytest.mark.parametrize("variant", list(range(P.variant_count())))
def test_each_variant_owns_every_node(variant):
    """Force one kernel variant to own every node of the DAG (all bins point
    to it) on graphs whose out-degrees it can hold."""
    cap = P.variant_capacity(variant)
    cases = [F.disjoint_union(F.complete(min(cap + 1, 18) if cap < 1000 else 40), F.wheel(20), F.windmill(6))]
    s, d = I.er(3000, 12000, variant + 1)
    cases.append((3000, s, d))  # max d+ stays small
    if cap >= 64:
        n, s, d = I.rmat(13, 16, seed=200 + variant)
        cases.append((n, s, d))
    if cap >= 300:
        n, s, d = I.rmat(16, 16, seed=300 + variant)
        cases.append((n, s, d))
    if cap >= 4096 or cap > 10**6:
        cases.append(F.complete(300))
    for n, s, d in cases:
        ref = oracle.count(n, s, d, order=1)
        r = gpu_count(n, s, d)
        if r["info"]["max_outdeg"] > cap:
            continue
        r = gpu_count(n, s, d, tuning=_tuning_all_to(variant))
        assert sum(r["info"]["bin_count"]) == r["info"]["bin_count"][N.NUM_BINS - 1]
        check_against(r, ref, n)


def test_hubs_above_every_table():
    """K_4200: nodes 0..102 have d+ above the largest LDS table (4096), so the
    default tuning sends them to the hub variant (a bitmap of N+(u) over all
    ids); then the same with the binary-search fallback. Closed form:
    T(v) = C(n-1, 2), CC = 1."""
    n = 4200
    iu = np.triu_indices(n, 1)
    s, d = iu[0].astype(np.int32), iu[1].astype(np.int32)
    g = P.Graph(n, to_dev(s), to_dev(d))
    assert g.info["max_outdeg"] == n - 1 and g.info["bin_count"][N.NUM_BINS - 1] == n - 1 - 4096
    for var in (P.default_tuning().bin_variant[N.NUM_BINS - 1], 8):
        t = P.default_tuning()
        t.bin_variant[N.NUM_BINS - 1] = var
        g.retune(t)
        for _ in range(2):  # the hub bitmaps are left clean for the next launch
            o = g.count()
            torch.cuda.synchronize()
            T = o["T"].cpu().numpy().view(np.uint64)
            assert np.all(T == (n - 1) * (n - 2) // 2), var
            assert int(o["total"].cpu().numpy().view(np.uint64)[0]) == n * (n - 1) * (n - 2) // 6
            assert np.all(o["cc"].cpu().numpy() == 1.0)


def test_cuckoo_tables_fall_back_to_buckets():
    """Cuckoo-table variants rebuild a node's table in the bucket layout when
    an insert gives up. Forced two ways: (1) K_5 on ids whose low 24 bits
    agree, so four keys share one slot pair; (2) K_4097 on the d+ <= 4096
    variant, whose largest tables are half full. Closed forms: T(v) =
    C(d(v), 2) on complete graphs, 0 elsewhere."""
    hub = [0, 1, 1 + (1 << 24), 1 + (1 << 25), 1 + 3 * (1 << 24)]
    n = hub[-1] + 1
    s = np.array([a for i, a in enumerate(hub) for b in hub[i + 1:]], dtype=np.int32)
    d = np.array([b for i, a in enumerate(hub) for b in hub[i + 1:]], dtype=np.int32)
    g = P.Graph(n, to_dev(s), to_dev(d))
    for var in (10, 11, 12, 13):
        g.retune(_tuning_all_to(var))
        o = g.count()
        torch.cuda.synchronize()
        T = o["T"].cpu().numpy().view(np.uint64)
        assert np.all(T[hub] == 6) and int(T.sum()) == 30, var
    k = 4097
    iu = np.triu_indices(k, 1)
    s, d = iu[0].astype(np.int32), iu[1].astype(np.int32)
    g = P.Graph(k, to_dev(s), to_dev(d))
    assert g.info["max_outdeg"] == k - 1
    for tun in (_tuning_all_to(14),
                {"bin_limit": [16, 64, 256, 1024, 4096], "bin_variant": [10, 11, 12, 13, 14, 9], "min_side": 1}):
        g.retune(tun)
        o = g.count()
        torch.cuda.synchronize()
        T = o["T"].cpu().numpy().view(np.uint64)
        assert np.all(T == (k - 1) * (k - 2) // 2)
        assert int(o["total"].cpu().numpy().view(np.uint64)[0]) == k * (k - 1) * (k - 2) // 6


def test_retune_matches():
    n, s, d = I.rmat(14, 16, seed=17)
    ref = oracle.count(n, s, d, order=1)
    g = P.Graph(n, to_dev(s), to_dev(d))
    for var in (2, 5, 8, P.variant_count() - 1):
        g.retune(_tuning_all_to(var) if P.variant_capacity(var) >= g.info["max_outdeg"] else P.default_tuning())
        o = g.count()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o["T"].cpu().numpy().view(np.uint64), ref["T"])


@pytest.mark.parametrize("tun", [
    {"bin_limit": [16, 16, 16, 16, 64], "bin_variant": [0, 0, 0, 0, 1, 8], "min_side": 1},
    {"bin_limit": [8, 24, 64, 256, 1024], "bin_variant": [21, 21, 21, 12, 13, 8], "min_side": 1},
    {"bin_limit": [4, 8, 32, 128, 256], "bin_variant": [10, 10, 11, 12, 12, 8], "min_side": 0},
])
def test_count_bins_merged_launches(tun):
    """Runs of adjacent bins with one variant launched as one grid
    (tricc_count_bins, as tricc_count issues them) give the oracle's T and
    total; ranges that mix variants or leave the bins are rejected."""
    n, s, d = I.rmat(15, 16, seed=47)
    ref = oracle.count(n, s, d, order=1)
    g = P.Graph(n, to_dev(s), to_dev(d), tuning=tun)
    L, h = N.lib(), g._h
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    T = torch.empty(n, dtype=torch.int64, device=DEV)
    cc = torch.empty(n, dtype=torch.float32, device=DEV)
    tot = torch.empty(1, dtype=torch.int64, device=DEV)
    avg = torch.empty(1, dtype=torch.float64, device=DEV)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    var = tun["bin_variant"]
    N.check(L.tricc_count_begin(h, ptr(T), sp), "begin")
    b0, launches = 0, 0
    while b0 < N.NUM_BINS:
        b1 = b0
        while b1 + 1 < N.NUM_BINS and var[b1 + 1] == var[b0]:
            b1 += 1
        N.check(L.tricc_count_bins(h, b0, b1, ptr(T), sp), "bins")
        launches += 1
        b0 = b1 + 1
    assert launches < N.NUM_BINS
    N.check(L.tricc_count_finish(h, ptr(T), ptr(cc), ptr(tot), ptr(avg), sp), "finish")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(T.cpu().numpy().view(np.uint64), ref["T"])
    assert int(tot.cpu().numpy().view(np.uint64)[0]) == ref["total"]
    mixed = next(b for b in range(N.NUM_BINS - 1) if var[b] != var[b + 1])
    for first, last in ((mixed, mixed + 1), (-1, 0), (0, N.NUM_BINS), (2, 1)):
        assert L.tricc_count_bins(h, first, last, ptr(T), sp) == N.TRICC_EINVAL


def test_tuning_capacity_violation_is_rejected():
    n, s, d = I.rmat(12, 16, seed=19)
    g = P.Graph(n, to_dev(s), to_dev(d))
    assert g.info["max_outdeg"] > 16
    with pytest.raises(N.TriccError) as ei:
        g.retune(_tuning_all_to(0))
    assert ei.value.status == N.TRICC_EINVAL
    # the previous tuning stays in force
    o = g.count()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o["T"].cpu().numpy().view(np.uint64), oracle.count(n, s, d)["T"])


def test_long_rows_take_every_sort_path():
    """A hub row above the LDS capacity (chunk sort + merge passes), rows in
    the 4k..32k LDS class, and heavy duplication inside long rows."""
    rng = np.random.default_rng(23)
    n = 120_000
    hub_leaves = rng.choice(np.arange(1, n), size=100_000, replace=False)
    s = [np.zeros(100_000, np.int64), np.full(9000, 1, np.int64), np.full(20000, 2, np.int64)]
    d = [hub_leaves, rng.integers(3, n, 9000), rng.integers(3, 3000, 20000)]  # node 2: many duplicates
    # duplicate part of the hub row, and random edges among leaves
    s.append(np.zeros(30_000, np.int64))
    d.append(hub_leaves[:30_000])
    s.append(rng.integers(1, n, 200_000))
    d.append(rng.integers(1, n, 200_000))
    s = np.concatenate(s).astype(np.int32)
    d = np.concatenate(d).astype(np.int32)
    perm = rng.permutation(s.size)
    r, ref = parity(n, s[perm], d[perm])
    assert r["info"]["large_rows"] >= 1
    assert r["info"]["max_deg"] >= 100_000


def test_sort_class_boundaries():
    """Hub rows whose raw lengths sit on both sides of every sort-class limit
    (1,024 / 4,096 / 8,192 / 16,384 / 32,768) and inside classes where the
    network spans fewer ids than the block holds; leaves drawn with
    replacement, so every long row also carries duplicates."""
    rng = np.random.default_rng(31)
    n = 60_000
    lengths = [1024, 1025, 1500, 2048, 2049, 4096, 4097, 5000, 8192, 8193, 9000, 16384, 16385, 32768, 32769]
    s = [np.full(L, h, np.int64) for h, L in enumerate(lengths)]
    d = [rng.integers(100, n, L) for L in lengths]
    hub_rows = [np.unique(x) for x in d]
    s.append(rng.integers(100, n, 100_000))
    d.append(rng.integers(100, n, 100_000))
    s = np.concatenate(s).astype(np.int32)
    d = np.concatenate(d).astype(np.int32)
    perm = rng.permutation(s.size)
    r, ref = parity(n, s[perm], d[perm])
    A = {k: v.cpu().numpy() for k, v in r["graph"].arrays().items()}
    for h, want in enumerate(hub_rows):
        np.testing.assert_array_equal(A["adj"][A["off"][h]:A["off"][h] + A["deg"][h]], want)
    assert r["info"]["large_rows"] >= 1


def test_partition_spread_over_several_blocks():
    """The raw rows are built per id range (1024 ids here); a range with more
    entries than one block takes (2^18) is split over blocks that combine
    their row lengths and cursors. Two hubs share the first range; edges
    straddle range boundaries; self loops and duplicates are mixed in."""
    rng = np.random.default_rng(31)
    n = 700_000
    hub_a = rng.choice(np.arange(1024, n), size=600_000, replace=False)
    hub_b = rng.choice(np.arange(1024, n), size=150_000, replace=False)
    b = np.arange(1024, n, 1024)
    s = [np.full(600_000, 5), np.full(150_000, 1000), hub_a[:40_000], rng.integers(0, n, 300_000), b - 1,
         np.arange(0, n, 997)]
    d = [hub_a, hub_b, np.full(40_000, 5), rng.integers(0, n, 300_000), b, np.arange(0, n, 997)]
    s = np.concatenate(s).astype(np.int32)
    d = np.concatenate(d).astype(np.int32)
    perm = rng.permutation(s.size)
    r, ref = parity(n, s[perm], d[perm])
    assert r["info"]["max_deg"] >= 600_000
    assert ref["deg"][5] >= 600_000


def test_build_beyond_partitioned_range():
    """More ids than the per-range build covers (4096 ranges of 2^14 ids):
    the build takes the per-entry path. Small components sit at both ends
    and in the middle of a 70M-id range."""
    n = 70_000_000
    comps = [(0, F.complete(6)), (35_000_000, F.wheel(9)), (n - 40, F.windmill(5)), (n - 12, F.complete(12))]
    s = np.concatenate([c[1] + o for o, c in comps]).astype(np.int32)
    d = np.concatenate([c[2] + o for o, c in comps]).astype(np.int32)
    r, ref = parity(n, s, d)
    assert r["total"] == 20 + 9 + 5 + 220


def _csr_of(n, s, d):
    """Host CSR whose row v lists w for every pair (v, w), in input order."""
    order = np.argsort(s, kind="stable")
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, s.astype(np.int64) + 1, 1)
    return np.cumsum(rowptr), d[order].astype(np.int32)


def to_dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to(DEV)


def test_from_csr_trusted_rows_match_pair_build():
    """A simple, sorted, symmetric CSR (the one the pair build produces) taken
    as it is: same counts, same arrays, no sort."""
    n, s, d = I.rmat(12, 16, seed=41)
    ref = oracle.count(n, s, d)
    g0 = P.Graph(n, to_dev(s), to_dev(d))
    A = {k: v.cpu().numpy() for k, v in g0.arrays().items()}
    rows = [A["adj"][A["off"][v]:A["off"][v] + A["deg"][v]] for v in range(n)]
    rowptr = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.concatenate(rows).astype(np.int32)
    g = P.Graph.from_csr(n, to_dev64(rowptr), to_dev(col), assume_simple_sorted_symmetric=True)
    o = g.count()
    torch.cuda.synchronize()
    r = {"T": o["T"].cpu().numpy().view(np.uint64), "cc": o["cc"].cpu().numpy(),
         "total": int(o["total"].cpu().numpy().view(np.uint64)[0]), "avg": float(o["avg"].item()), "info": g.info,
         "check": g.count_check()}
    check_against(r, ref, n)
    B = {k: v.cpu().numpy() for k, v in g.arrays().items()}
    np.testing.assert_array_equal(B["deg"], A["deg"])
    np.testing.assert_array_equal(B["doff"], A["doff"])
    np.testing.assert_array_equal(B["dcol"], A["dcol"])
    assert g.info["n_deg2"] == int((ref["deg"] >= 2).sum()) == g0.info["n_deg2"]


def test_from_csr_general_rows_take_the_full_build():
    """Rows in any order with duplicates, self loops and one-sided entries:
    every entry is a pair (v, w)."""
    n, s, d = F.messy(*I.rmat(11, 8, seed=43), seed=44)
    rowptr, col = _csr_of(n, s, d)
    ref = oracle.count(n, s, d)
    g = P.Graph.from_csr(n, to_dev64(rowptr), to_dev(col))
    o = g.count()
    torch.cuda.synchronize()
    r = {"T": o["T"].cpu().numpy().view(np.uint64), "cc": o["cc"].cpu().numpy(),
         "total": int(o["total"].cpu().numpy().view(np.uint64)[0]), "avg": float(o["avg"].item()), "info": g.info,
         "check": g.count_check()}
    check_against(r, ref, n)
    # empty graph and isolated ids
    g = P.Graph.from_csr(5, to_dev64(np.zeros(6, np.int64)), to_dev(np.zeros(0, np.int32)), True)
    assert g.count()["total"].item() == 0 and g.info["n_deg2"] == 0


def test_from_csr_rejects_malformed_input():
    col = to_dev(np.array([1, 2, 0, 2, 0, 1], np.int32))
    good = np.array([0, 2, 4, 6], np.int64)
    assert P.Graph.from_csr(3, to_dev64(good), col, True).info["m"] == 3
    for bad in ([0, 3, 2, 6], [1, 2, 4, 6], [0, 2, 4, 5]):
        for trusted in (False, True):
            with pytest.raises(N.TriccError) as ei:
                P.Graph.from_csr(3, to_dev64(np.array(bad, np.int64)), col, trusted)
            assert ei.value.status == N.TRICC_EINVAL, (bad, trusted)
    with pytest.raises(N.TriccError) as ei:  # row 0 not ascending
        P.Graph.from_csr(3, to_dev64(good), to_dev(np.array([2, 1, 0, 2, 0, 1], np.int32)), True)
    assert ei.value.status == N.TRICC_EINVAL
    with pytest.raises(N.TriccError) as ei:  # self loop in a trusted row
        P.Graph.from_csr(3, to_dev64(good), to_dev(np.array([0, 2, 0, 2, 0, 1], np.int32)), True)
    assert ei.value.status == N.TRICC_EINVAL
    for trusted in (False, True):
        with pytest.raises(N.TriccError) as ei:
            P.Graph.from_csr(3, to_dev64(good), to_dev(np.array([1, 2, 0, 7, 0, 1], np.int32)), trusted)
        assert ei.value.status == N.TRICC_ERANGE

"""Seeded generators: determinism and the structural facts each promises."""
import math

import numpy as np
import pytest

from paper_1606_07550_amd import inputs as I


def test_er_exact_pairs_and_determinism():
    s, d = I.er(10_000, 100_000, 1)
    s2, d2 = I.er(10_000, 100_000, 1)
    np.testing.assert_array_equal(s, s2)
    np.testing.assert_array_equal(d, d2)
    assert np.all(s != d)
    key = np.minimum(s, d).astype(np.int64) * 10_000 + np.maximum(s, d)
    assert np.unique(key).size == 100_000
    assert s.min() >= 0 and max(s.max(), d.max()) < 10_000
    s3, _ = I.er(10_000, 100_000, 2)
    assert not np.array_equal(s, s3)
    # full graph: every pair exactly once
    s, d = I.er(30, 435, 5)
    key = np.minimum(s, d).astype(np.int64) * 30 + np.maximum(s, d)
    assert np.unique(key).size == 435
    with pytest.raises(ValueError):
        I.er(30, 436, 5)


def test_rmat_marginals():
    n, s, d = I.rmat(16, 16, seed=3, permute=False)
    assert n == 1 << 16 and s.size == 16 << 16
    top_s = (s >> 15) & 1
    top_d = (d >> 15) & 1
    # P(src bit = 1) = c + d = 0.24, P(dst bit = 1) = b + d = 0.24 (noise is symmetric)
    assert abs(top_s.mean() - 0.24) < 0.01
    assert abs(top_d.mean() - 0.24) < 0.01
    assert abs((top_s & top_d).mean() - 0.05) < 0.005
    n2, s2, d2 = I.rmat(16, 16, seed=3, permute=True)
    # the permutation is a bijection: degree multisets agree
    dg = np.bincount(np.concatenate([s, d]), minlength=n)
    dg2 = np.bincount(np.concatenate([s2, d2]), minlength=n)
    np.testing.assert_array_equal(np.sort(dg), np.sort(dg2))
    _, s3, d3 = I.rmat(16, 16, seed=3, permute=True)
    np.testing.assert_array_equal(s2, s3)


def test_ba_structure():
    n, k = 500, 4
    s, d = I.ba(n, k, 9)
    assert s.size == k * (k + 1) // 2 + (n - k - 1) * k
    key = np.minimum(s, d).astype(np.int64) * n + np.maximum(s, d)
    assert np.unique(key).size == s.size  # distinct targets, no repeats
    assert np.all(s != d)
    deg = np.bincount(np.concatenate([s, d]), minlength=n)
    assert deg.sum() == 2 * s.size and deg.min() >= k


def test_batch_sizes():
    b = I.batch(256, 4096)
    assert b["n"].min() >= 64 and b["n"].max() <= 65536
    fam = b["family"]
    assert 0.35 < fam.mean() < 0.65
    for g in range(0, 256, 17):
        e0, e1 = b["edge_off"][g], b["edge_off"][g + 1]
        s, d = b["src"][e0:e1], b["dst"][e0:e1]
        n = b["n"][g]
        assert s.size == b["m"][g]
        if s.size:
            assert s.min() >= 0 and max(s.max(), d.max()) < n
        if fam[g] == 1:
            assert 4 <= b["param"][g] <= 32
        else:
            assert 2 <= b["param"][g] <= 16
    b2 = I.batch(256, 4096)
    np.testing.assert_array_equal(b["src"], b2["src"])
    # log-uniform sizes: median near sqrt(64 * 65536)
    big = I.batch(2000, 7)
    assert 1200 < np.median(big["n"]) < 3300


def test_bfs_balls():
    n, s, d = I.rmat(12, 8, seed=5)
    off, nodes, seeds = I.bfs_queries(n, s, d, 40, seed=6, kmin=16, kmax=2000)
    k_req = I.query_sizes(40, 6, 16, 2000)
    adj = [set() for _ in range(n)]
    for a, b in zip(s.tolist(), d.tolist()):
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    for q in range(40):
        S = nodes[off[q]:off[q + 1]]
        assert S.size <= k_req[q] and S.size >= 1
        assert S[0] == seeds[q]
        assert np.unique(S).size == S.size
        seen = {int(S[0])}
        for x in S[1:]:
            assert adj[int(x)] & seen  # attached to an earlier ball node
            seen.add(int(x))
    assert np.all(np.log(k_req) >= math.log(16) - 1e-9)


def test_poisson_mean():
    t = I.poisson_arrivals(20000, 50.0, 1)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 50.0) < 0.001

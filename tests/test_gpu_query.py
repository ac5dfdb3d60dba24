"""GPU parity of the edge-existence tests (tricc_graph_has_edges) against the
oracle's search in the sorted edge set: every pair of small graphs (and ids
outside [0, n)), mixed true and random queries on R-MAT and on the paper's
smallest edge-test configuration (G(n=1M, m=10M), one random query per
edge), graphs built from edge lists and from a CSR, and the call's error
paths. Results are uint8 codes, compared exactly."""
import ctypes

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def gpu_has(g, qu, qv):
    out = g.has_edges(dev(qu), dev(qv))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def all_pairs(n):
    qu, qv = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    bad_u = np.array([-1, n, 0, n + 5, -7, 2**31 - 1])
    bad_v = np.array([0, 0, n, 1, -1, 0])
    return (np.concatenate([qu.ravel(), bad_u]).astype(np.int32),
            np.concatenate([qv.ravel(), bad_v]).astype(np.int32))


def mixed_queries(n, s, d, k, seed):
    """k queries: half input pairs in a random direction, half random pairs."""
    rng = np.random.default_rng(seed)
    h = k // 2
    e = rng.integers(0, s.size, h)
    flip = rng.integers(0, 2, h).astype(bool)
    qu = np.concatenate([np.where(flip, d[e], s[e]), rng.integers(0, n, k - h)]).astype(np.int32)
    qv = np.concatenate([np.where(flip, s[e], d[e]), rng.integers(0, n, k - h)]).astype(np.int32)
    return qu, qv


SMALL = [
    ("messy_K8", lambda: F.messy(*F.complete(8), seed=3)),
    ("wheel", lambda: F.wheel(17)),
    ("star", lambda: F.star(25)),
    ("windmill", lambda: F.windmill(6)),
    ("rmat8", lambda: I.rmat(8, 8, seed=4)),
    ("er", lambda: (60, *I.er(60, 400, 5))),
    ("loops_only", lambda: (5, np.array([0, 1, 2], np.int32), np.array([0, 1, 2], np.int32))),
    ("no_edges", lambda: (7, np.zeros(0, np.int32), np.zeros(0, np.int32))),
]


@pytest.mark.parametrize("name", [c[0] for c in SMALL])
def test_every_pair_of_small_graphs(name):
    n, s, d = dict(SMALL)[name]()
    qu, qv = all_pairs(n)
    g = P.Graph(n, dev(s), dev(d))
    np.testing.assert_array_equal(gpu_has(g, qu, qv), oracle.has_edges(n, s, d, qu, qv))


def test_rmat16_true_random_and_hub_queries():
    n, s, d = I.rmat(16, 16, seed=31)
    g = P.Graph(n, dev(s), dev(d))
    qu, qv = mixed_queries(n, s, d, 1 << 20, 32)
    # the largest hub against every id, both ways round
    hub = int(np.argmax(g.arrays()["deg"].cpu().numpy()))
    ids = np.arange(n, dtype=np.int32)
    qu = np.concatenate([qu, np.full(n, hub, np.int32), ids])
    qv = np.concatenate([qv, ids, np.full(n, hub, np.int32)])
    got = gpu_has(g, qu, qv)
    ref = oracle.has_edges(n, s, d, qu, qv)
    np.testing.assert_array_equal(got, ref)
    first = slice(0, 1 << 19)
    assert got[first][qu[first] != qv[first]].all()  # every input pair but a loop is an edge


def test_graph_from_csr_and_edge_list_agree():
    n, s, d = I.rmat(12, 16, seed=33)
    a = np.minimum(s, d).astype(np.int64)
    b = np.maximum(s, d).astype(np.int64)
    keep = a != b
    key = np.unique(a[keep] * n + b[keep])
    u, v = key // n, key % n
    rows = np.concatenate([u, v])
    cols = np.concatenate([v, u])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    g = P.Graph.from_csr(n, torch.from_numpy(rowptr).to(DEV), dev(cols), assume_simple_sorted_symmetric=True)
    qu, qv = mixed_queries(n, s, d, 200000, 34)
    np.testing.assert_array_equal(gpu_has(g, qu, qv), oracle.has_edges(n, s, d, qu, qv))


def test_paper_config_er_1m_10m():
    """G(n=1M, m=10M) with one random query per edge (Section 6.2's smallest
    edge-test graph), plus every input pair."""
    n, m = 1_000_000, 10_000_000
    s, d = I.er(n, m, 35)
    g = P.Graph(n, dev(s), dev(d))
    rng = np.random.default_rng(36)
    qu = np.concatenate([rng.integers(0, n, m), s]).astype(np.int32)
    qv = np.concatenate([rng.integers(0, n, m), d]).astype(np.int32)
    got = gpu_has(g, qu, qv)
    np.testing.assert_array_equal(got, oracle.has_edges(n, s, d, qu, qv))
    assert got[m:].all()


def test_empty_queries_and_errors():
    n, s, d = F.complete(6)
    g = P.Graph(n, dev(s), dev(d))
    e = torch.empty(0, dtype=torch.int32, device=DEV)
    assert g.has_edges(e, e).numel() == 0
    L = N.lib()
    assert L.tricc_graph_has_edges(None, 1, None, None, None, None) == N.TRICC_EINVAL
    assert L.tricc_graph_has_edges(g._h, -1, None, None, None, None) == N.TRICC_EINVAL
    assert L.tricc_graph_has_edges(g._h, 4, None, None, None, None) == N.TRICC_EINVAL
    assert L.tricc_graph_has_edges(g._h, 0, None, None, None, None) == N.TRICC_OK
    with pytest.raises(ValueError):
        g.has_edges(dev([0, 1]), torch.zeros(2, dtype=torch.int64, device=DEV))
    # results do not depend on the stream or on a count running before them
    qu, qv = all_pairs(n)
    o = g.count()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        out = g.has_edges(dev(qu), dev(qv), stream=side)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.has_edges(n, s, d, qu, qv))
    assert int(o["total"].cpu().numpy().view(np.uint64)[0]) == 20

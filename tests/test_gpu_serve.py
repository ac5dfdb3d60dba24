"""GPU parity of the query server: each query's triangle count and average
clustering coefficient of G[S] against the oracle's induced-subgraph
definition; results identical alone and in a mix; admission by memory."""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1606_07550_amd as P
from paper_1606_07550_amd import _native as N
from paper_1606_07550_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CC_RTOL = 1e-6


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


@pytest.fixture(scope="module")
def resident():
    n, s, d = I.rmat(13, 16, seed=21)
    g = P.Graph(n, dev(s), dev(d))
    off, nodes, _ = I.bfs_queries(n, s, d, 24, seed=22, kmin=16, kmax=3000)
    queries = [nodes[off[q]:off[q + 1]] for q in range(24)]
    rng = np.random.default_rng(23)
    queries.append(rng.choice(n, size=500, replace=False).astype(np.int32))  # scattered set
    queries.append(np.arange(n, dtype=np.int32))  # G[V] = G
    queries.append(np.array([5], np.int32))
    return n, s, d, g, queries


def collect(srv, nq, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < nq:
        for r in srv.poll():
            out[r["qid"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError("server results missing")
        time.sleep(0.001)
    return out


def test_queries_match_oracle(resident):
    n, s, d, g, queries = resident
    srv = P.Server(g, 1 << 30, slots=2)
    for q, S in enumerate(queries):
        assert srv.submit(q, S) == N.TRICC_OK
    srv.drain()
    res = collect(srv, len(queries))
    full = oracle.count(n, s, d)
    for q, S in enumerate(queries):
        r = res[q]
        assert r["status"] == 0
        ref = oracle.induced(n, s, d, S)
        assert r["triangles"] == ref["total"], q
        assert r["m"] == ref["m"], q
        assert abs(r["avg_cc"] - ref["avg"]) <= CC_RTOL * abs(ref["avg"]), q
    # G[V] = G
    r = res[len(queries) - 2]
    assert r["triangles"] == full["total"]
    srv.close()


def test_alone_equals_mixed(resident):
    n, s, d, g, queries = resident
    srv = P.Server(g, 1 << 30, slots=3, max_batch_queries=64)
    alone = {}
    for q, S in enumerate(queries):
        srv.submit(q, S)
        srv.drain()
        alone.update(collect(srv, 1))
    order = np.random.default_rng(5).permutation(len(queries))
    for q in order:
        srv.submit(int(q) + 1000, queries[q])
    srv.drain()
    mixed = collect(srv, len(queries))
    assert max(r["batch_size"] for r in mixed.values()) > 1  # queries really shared batches
    for q in range(len(queries)):
        a, b = alone[q], mixed[q + 1000]
        assert a["triangles"] == b["triangles"]
        assert a["avg_cc"] == b["avg_cc"]  # bit-identical
        assert a["m"] == b["m"]
    srv.close()


def test_admission_by_memory(resident):
    n, s, d, g, queries = resident
    big = queries[len(queries) - 2]  # all nodes
    probe = P.Server(g, 1 << 30, slots=1)
    need = probe.query_bytes(big)
    probe.close()
    # room for exactly one such query at a time
    srv = P.Server(g, int(need * 1.5), slots=1)
    assert srv.submit(1, big) == N.TRICC_OK
    rc = srv.submit(2, big)
    if rc == N.TRICC_EBUSY:
        srv.drain()
        assert srv.submit(2, big) == N.TRICC_OK
    srv.drain()
    res = collect(srv, 2)
    assert res[1]["triangles"] == res[2]["triangles"]
    srv.close()
    # a query that can never fit a slot
    tiny = P.Server(g, need // 4, slots=1)
    with pytest.raises(N.TriccError) as ei:
        tiny.submit(3, big)
    assert ei.value.status == N.TRICC_ENOMEM
    tiny.close()


def test_bad_queries_rejected(resident):
    n, s, d, g, queries = resident
    srv = P.Server(g, 1 << 28, slots=1)
    with pytest.raises(N.TriccError) as ei:
        srv.submit(1, np.array([1, 2, 1], np.int32))
    assert ei.value.status == N.TRICC_EINVAL
    with pytest.raises(N.TriccError) as ei:
        srv.submit(2, np.array([1, n], np.int32))
    assert ei.value.status == N.TRICC_ERANGE
    assert srv.submit(3, np.zeros(0, np.int32)) == N.TRICC_OK
    srv.drain()
    r = collect(srv, 1)[3]
    assert r["k"] == 0 and r["triangles"] == 0 and r["avg_cc"] == 0.0
    srv.close()


@pytest.mark.parametrize("tun", [
    {"merge_limit": 16, "wave_limit": 64, "persist_variant": 2, "blocks_per_cu": 0},
    {"merge_limit": 4, "wave_limit": 32, "persist_variant": 3, "blocks_per_cu": 1},
    {"merge_limit": 32, "wave_limit": 64, "persist_variant": 1, "blocks_per_cu": 0},
    {"merge_limit": 0, "wave_limit": 64, "persist_variant": 0, "blocks_per_cu": 0},
    {"merge_limit": 16, "wave_limit": 64, "persist_variant": 6, "blocks_per_cu": 0},
])
def test_every_batch_variant_serves(resident, tun):
    n, s, d, g, queries = resident
    srv = P.Server(g, 1 << 30, slots=2)
    srv.set_tuning(tun)
    picks = list(range(6)) + [len(queries) - 3]
    for q in picks:
        assert srv.submit(q, queries[q]) == N.TRICC_OK
    srv.drain()
    res = collect(srv, len(picks))
    for q in picks:
        ref = oracle.induced(n, s, d, queries[q])
        assert res[q]["status"] == 0 and res[q]["triangles"] == ref["total"], (tun, q)
    with pytest.raises(Exception):
        srv.set_tuning({"merge_limit": 17, "wave_limit": 64, "persist_variant": 2, "blocks_per_cu": 0})
    srv.close()

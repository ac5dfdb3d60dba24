"""GPU parity of the batched path: per-graph results against the oracle run
on each graph alone; hipGraph replays against eager launches; batched
against single-graph results; every persistent variant and work split."""
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


def pack(graphs):
    """[(n, src, dst)] -> node_off, edge_off, src, dst (local ids)."""
    node_off = np.zeros(len(graphs) + 1, np.int64)
    edge_off = np.zeros(len(graphs) + 1, np.int64)
    for i, (n, s, d) in enumerate(graphs):
        node_off[i + 1] = node_off[i] + n
        edge_off[i + 1] = edge_off[i] + len(s)
    src = np.concatenate([g[1] for g in graphs]).astype(np.int32) if graphs else np.zeros(0, np.int32)
    dst = np.concatenate([g[2] for g in graphs]).astype(np.int32) if graphs else np.zeros(0, np.int32)
    return node_off, edge_off, src, dst


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(DEV)


def to_host(out):
    return {
        "T": out["T"].cpu().numpy().view(np.uint64),
        "cc": out["cc"].cpu().numpy(),
        "graph_tri": out["graph_tri"].cpu().numpy().view(np.uint64),
        "graph_avg": out["graph_avg"].cpu().numpy(),
        "batch_tri": int(out["batch_tri"].cpu().numpy().view(np.uint64)[0]),
    }


def check_batch(r, graphs, node_off):
    # the batch total comes from the intersection kernels' own counters, the
    # per-graph totals from the per-node counts
    assert r["batch_tri"] == int(r["graph_tri"].sum(dtype=np.uint64))
    for gi, (n, s, d) in enumerate(graphs):
        ref = oracle.count(n, s, d)
        a, b = node_off[gi], node_off[gi + 1]
        np.testing.assert_array_equal(r["T"][a:b], ref["T"], err_msg=f"graph {gi}")
        assert r["graph_tri"][gi] == ref["total"], gi
        np.testing.assert_allclose(r["cc"][a:b].astype(np.float64), ref["cc"], rtol=CC_RTOL, atol=0)
        assert np.array_equal(r["cc"][a:b] == 0, ref["cc"] == 0)
        assert abs(r["graph_avg"][gi] - ref["avg"]) <= CC_RTOL * abs(ref["avg"]), gi


def mixed_graphs():
    b = I.batch(48, 77, nmin=64, nmax=3000)
    graphs = []
    for g in range(48):
        e0, e1 = b["edge_off"][g], b["edge_off"][g + 1]
        graphs.append((int(b["n"][g]), b["src"][e0:e1], b["dst"][e0:e1]))
    graphs += [F.complete(300), F.wheel(40), F.star(500), (7, np.zeros(0, np.int32), np.zeros(0, np.int32)),
               (0, np.zeros(0, np.int32), np.zeros(0, np.int32)), F.messy(*F.windmill(9), seed=3)]
    n, s, d = I.rmat(12, 16, seed=5)
    graphs.append((n, s, d))
    return graphs


@pytest.fixture(scope="module")
def mixed():
    graphs = mixed_graphs()
    return graphs, pack(graphs)


def test_batch_matches_oracle(mixed):
    graphs, (node_off, edge_off, src, dst) = mixed
    print(f"[batch] G={len(graphs)} nodes={node_off[-1]} pairs={edge_off[-1]}", flush=True)
    b = P.Batch(node_off, edge_off, dev(src), dev(dst))
    info = b.info
    assert info["hub_nodes"] > 0  # K_300 has out-degrees above 256
    b.plan()
    b.run()
    torch.cuda.synchronize()
    check_batch(to_host(b.out), graphs, node_off)


def test_graph_replays_match_eager(mixed):
    graphs, (node_off, edge_off, src, dst) = mixed
    b = P.Batch(node_off, edge_off, dev(src), dev(dst))
    b.plan()
    b.run_eager()
    torch.cuda.synchronize()
    ref = to_host(b.out)
    scratch = torch.zeros(1 << 20, device=DEV)
    for rep in range(4):
        scratch.add_(1.0)  # unrelated eager work between replays
        b.out["T"].fill_(7)
        b.out["graph_avg"].fill_(-1.0)
        b.run()
        torch.cuda.synchronize()
        r = to_host(b.out)
        for k in ref:
            np.testing.assert_array_equal(r[k], ref[k], err_msg=f"replay {rep} field {k}")


@pytest.mark.parametrize("tun", [
    {"merge_limit": 0, "wave_limit": 64, "persist_variant": 0, "blocks_per_cu": 0},
    {"merge_limit": 0, "wave_limit": 16, "persist_variant": 0, "blocks_per_cu": 1},
    {"merge_limit": 2, "wave_limit": 2, "persist_variant": 1, "blocks_per_cu": 2},
    {"merge_limit": 40, "wave_limit": 40, "persist_variant": 1, "blocks_per_cu": 0},
    {"merge_limit": 64, "wave_limit": 64, "persist_variant": 0, "blocks_per_cu": 4},
    {"merge_limit": 8, "wave_limit": 32, "persist_variant": 0, "blocks_per_cu": 0},
    {"merge_limit": 16, "wave_limit": 64, "persist_variant": 2, "blocks_per_cu": 0},
    {"merge_limit": 16, "wave_limit": 32, "persist_variant": 3, "blocks_per_cu": 2},
    {"merge_limit": 3, "wave_limit": 8, "persist_variant": 2, "blocks_per_cu": 1},
    {"merge_limit": 32, "wave_limit": 64, "persist_variant": 4, "blocks_per_cu": 0},
    {"merge_limit": 8, "wave_limit": 64, "persist_variant": 5, "blocks_per_cu": 0},
    {"merge_limit": 16, "wave_limit": 64, "persist_variant": 6, "blocks_per_cu": 0},
    {"merge_limit": 5, "wave_limit": 24, "persist_variant": 7, "blocks_per_cu": 1},
])
def test_tunings_agree(mixed, tun):
    graphs, (node_off, edge_off, src, dst) = mixed
    b = P.Batch(node_off, edge_off, dev(src), dev(dst), tuning=tun)
    b.plan()
    b.run()
    torch.cuda.synchronize()
    check_batch(to_host(b.out), graphs, node_off)
    # retune back to the default and compare
    b.retune(P.default_batch_tuning())
    b.plan()
    b.run()
    torch.cuda.synchronize()
    check_batch(to_host(b.out), graphs, node_off)


def test_small_node_path_limit_is_enforced(mixed):
    graphs, (node_off, edge_off, src, dst) = mixed
    b = P.Batch(node_off, edge_off, dev(src), dev(dst))
    with pytest.raises(N.TriccError) as ei:
        b.retune({"merge_limit": 17, "wave_limit": 64, "persist_variant": 2, "blocks_per_cu": 0})
    assert ei.value.status == N.TRICC_EINVAL


def test_batched_equals_single_graph(mixed):
    graphs, (node_off, edge_off, src, dst) = mixed
    b = P.Batch(node_off, edge_off, dev(src), dev(dst))
    b.plan()
    b.run()
    torch.cuda.synchronize()
    r = to_host(b.out)
    for gi in (0, 5, 17, len(graphs) - 1):
        n, s, d = graphs[gi]
        g = P.Graph(n, dev(s), dev(d))
        o = g.count()
        torch.cuda.synchronize()
        a, e = node_off[gi], node_off[gi + 1]
        np.testing.assert_array_equal(o["T"].cpu().numpy().view(np.uint64), r["T"][a:e])
        np.testing.assert_array_equal(o["cc"].cpu().numpy(), r["cc"][a:e])
        assert int(o["total"].cpu().numpy().view(np.uint64)[0]) == r["graph_tri"][gi]
        assert abs(o["avg"].item() - r["graph_avg"][gi]) <= 1e-12 * max(1e-300, abs(r["graph_avg"][gi]))


def test_cuckoo_small_tables_fall_back_to_buckets():
    """A member with K_5 on local ids whose low 24 bits agree: four keys of
    one short-list node share a cuckoo slot pair, so that wave's tables are
    rebuilt in the bucket layout. Closed form: T = 6 on the K_5, 0 elsewhere;
    the other members against the oracle."""
    hub = [0, 1, 1 + (1 << 24), 1 + (1 << 25), 1 + 3 * (1 << 24)]
    pairs = [(a, b) for i, a in enumerate(hub) for b in hub[i + 1:]]
    big = (hub[-1] + 1, np.array([p[0] for p in pairs], np.int32), np.array([p[1] for p in pairs], np.int32))
    small = [F.complete(12), F.wheel(15), F.windmill(4)]
    graphs = small + [big]
    node_off, edge_off, src, dst = pack(graphs)
    for pv in (6, 7, 2):
        b = P.Batch(node_off, edge_off, dev(src), dev(dst),
                    tuning={"merge_limit": 16, "wave_limit": 64, "persist_variant": pv, "blocks_per_cu": 0})
        b.plan()
        b.run()
        torch.cuda.synchronize()
        r = to_host(b.out)
        check_batch(r, small, node_off)
        T = r["T"][node_off[3]:node_off[4]]
        assert np.all(T[hub] == 6) and int(T.sum()) == 30, pv
        assert r["graph_tri"][3] == 10, pv


def test_bad_local_id_is_rejected():
    graphs = [F.complete(5), (4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))]
    node_off, edge_off, src, dst = pack(graphs)
    with pytest.raises(N.TriccError) as ei:
        P.Batch(node_off, edge_off, dev(src), dev(dst))
    assert ei.value.status == N.TRICC_ERANGE


def test_empty_batch_members():
    graphs = [(0, np.zeros(0, np.int32), np.zeros(0, np.int32)), (3, np.zeros(0, np.int32), np.zeros(0, np.int32)),
              F.complete(4)]
    node_off, edge_off, src, dst = pack(graphs)
    b = P.Batch(node_off, edge_off, dev(src), dev(dst))
    b.plan()
    b.run()
    torch.cuda.synchronize()
    r = to_host(b.out)
    assert list(r["graph_tri"]) == [0, 0, 4]
    assert r["graph_avg"][0] == 0.0 and r["graph_avg"][1] == 0.0 and r["graph_avg"][2] == 1.0


def packed_csr(graphs, simple):
    """Packed CSR of the graphs (local ids): simple=True gives each graph's
    simple symmetric rows, ascending; False gives the raw pairs as rows
    (row u holds v for every input pair (u, v))."""
    rows, cols = [], []
    n0 = 0
    for n, s, d in graphs:
        s = s.astype(np.int64)
        d = d.astype(np.int64)
        if simple:
            a, b = np.minimum(s, d), np.maximum(s, d)
            keep = a != b
            key = np.unique(a[keep] * max(n, 1) + b[keep])
            u, v = key // max(n, 1), key % max(n, 1)
            r, c = np.concatenate([u, v]), np.concatenate([v, u])
        else:
            r, c = s, d
        o = np.lexsort((c, r))
        rows.append(r[o] + n0)
        cols.append(c[o])
        n0 += n
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols).astype(np.int32) if cols else np.zeros(0, np.int32)
    rowptr = np.zeros(n0 + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n0), out=rowptr[1:])
    return rowptr, cols


@pytest.mark.parametrize("simple", [True, False])
def test_packed_csr_batch_matches_oracle(mixed, simple):
    graphs, (node_off, edge_off, src, dst) = mixed
    rowptr, col = packed_csr(graphs, simple)
    print(f"[batch csr] simple={simple} G={len(graphs)} nnz={col.size}", flush=True)
    b = P.Batch.from_csr(node_off, torch.from_numpy(rowptr).to(DEV), dev(col), assume_simple_sorted_symmetric=simple)
    b.plan()
    b.run()
    torch.cuda.synchronize()
    check_batch(to_host(b.out), graphs, node_off)


def test_packed_csr_batch_errors(mixed):
    graphs = [F.complete(5), F.wheel(6)]
    node_off, _, _, _ = pack(graphs)
    rowptr, col = packed_csr(graphs, True)
    bad = col.copy()
    bad[-1] = 7  # the wheel has local ids 0..6: 7 is outside its range
    for simple in (True, False):
        with pytest.raises(N.TriccError) as ei:
            P.Batch.from_csr(node_off, torch.from_numpy(rowptr).to(DEV), dev(bad), assume_simple_sorted_symmetric=simple)
        assert ei.value.status == N.TRICC_ERANGE
    rp = rowptr.copy()
    rp[3], rp[4] = rp[4], rp[3]  # not non-decreasing
    with pytest.raises(N.TriccError) as ei:
        P.Batch.from_csr(node_off, torch.from_numpy(rp).to(DEV), dev(col), assume_simple_sorted_symmetric=True)
    assert ei.value.status in (N.TRICC_EINVAL, N.TRICC_ERANGE)

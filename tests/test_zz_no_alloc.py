"""The entry point that allocates nothing (tricc_count_noalloc, a fixed
device array as the graph workspace) against the allocating path
(tricc_graph_build + tricc_count) and the oracle, through the C ABI: two
calls in a row, the second on a smaller graph, so the second runs on the
array the first left behind."""
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


def noalloc(n, s, d):
    T = torch.full((max(n, 1),), -1, dtype=torch.int64, device=DEV)
    cc = torch.full((max(n, 1),), -1.0, dtype=torch.float32, device=DEV)
    tot = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    avg = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
    S, D = dev(s), dev(d)
    rc = N.lib().tricc_count_noalloc(n, S.numel(), ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(D.data_ptr()),
                                     ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(cc.data_ptr()),
                                     ctypes.c_void_p(tot.data_ptr()), ctypes.c_void_p(avg.data_ptr()), None)
    N.check(rc, "tricc_count_noalloc")
    torch.cuda.synchronize()
    return (T[:n].cpu().numpy().view(np.uint64), cc[:n].cpu().numpy(), int(tot.cpu().numpy().view(np.uint64)[0]),
            float(avg.item()))


def allocating(n, s, d):
    g = P.Graph(n, dev(s), dev(d))
    o = g.count()
    torch.cuda.synchronize()
    return (o["T"].cpu().numpy().view(np.uint64), o["cc"].cpu().numpy(), int(o["total"].cpu().numpy().view(np.uint64)[0]),
            float(o["avg"].item()))


def test_noalloc_matches_allocating_path_twice():
    # first the largest graph the array takes (65,536 ids, 2^20 pairs, an R-MAT
    # with a hub), then a smaller one on the same array
    n1, s1, d1 = I.rmat(16, 16, seed=91)
    s2, d2 = I.er(3000, 20000, 92)
    n2 = 3000
    for n, s, d in ((n1, s1, d1), (n2, s2, d2)):
        print(f"[noalloc] n={n} m_raw={s.size}", flush=True)
        a = noalloc(n, s, d)
        b = allocating(n, s, d)
        ref = oracle.count(n, s, d)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[0], ref["T"])
        np.testing.assert_array_equal(a[1], b[1])
        np.testing.assert_allclose(a[1].astype(np.float64), ref["cc"], rtol=1e-6, atol=0)
        assert a[2] == b[2] == ref["total"]
        assert a[3] == b[3] and abs(a[3] - ref["avg"]) <= 1e-6 * abs(ref["avg"])


def test_noalloc_small_cases_and_errors():
    for n, s, d in (F.complete(40), F.messy(*F.wheel(30), seed=4), (9, np.zeros(0, np.int32), np.zeros(0, np.int32))):
        a = noalloc(n, s, d)
        ref = oracle.count(n, s, d)
        np.testing.assert_array_equal(a[0], ref["T"])
        assert a[2] == ref["total"]
    with pytest.raises(N.TriccError) as ei:
        noalloc(5, np.array([0, 7], np.int32), np.array([1, 2], np.int32))
    assert ei.value.status == N.TRICC_ERANGE
    # a valid call after the error still gives the right result
    n, s, d = F.complete(12)
    assert noalloc(n, s, d)[2] == 220

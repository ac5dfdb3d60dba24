"""GPU parity of the device G(n, m) and Barabasi-Albert generators
(tricc_gen_er, tricc_gen_ba) against the oracle's generators of the same
definitions: every edge bit-exact at small and medium sizes (the G(10^4,
10^5) configuration among them, the largest batch member for BA), dense and
degenerate cases, repeat calls; at the edge-existence benchmark's size
G(10^7, 10^8) the first 2M edges against the oracle (the first m' edges of
G(n, m) are G(n, m') by definition) and the whole list for what holds at any
size (m distinct loop-free pairs); and the argument errors."""
import numpy as np
import pytest
import torch

import oracle
import paper_1606_07550_amd as P
from paper_1606_07550_amd import _native as N
from paper_1606_07550_amd import generators as GEN

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("n,m", [(2, 1), (3, 3), (9, 36), (300, 44850), (300, 20000), (1000, 1), (10_000, 100_000),
                                 (50_000, 1_000_000), (1_000_000, 10_000_000), (7, 0)])
@pytest.mark.parametrize("seed", [1, 2**64 - 1])
def test_er_against_oracle(n, m, seed):
    print(f"[gen er] n={n} m={m} seed={seed}", flush=True)
    s, d = GEN.er(n, m, seed=seed, device=DEV)
    torch.cuda.synchronize()
    s2, d2 = oracle.er(n, m, seed)
    assert np.array_equal(host(s), s2) and np.array_equal(host(d), d2)


def test_er_full_size_prefix_and_properties():
    n, m = 10_000_000, 100_000_000
    print(f"[gen er] full size n={n} m={m}", flush=True)
    s, d = GEN.er(n, m, seed=2016, device=DEV)
    torch.cuda.synchronize()
    k = 2_000_000
    s2, d2 = oracle.er(n, k, 2016)
    assert np.array_equal(host(s[:k]), s2) and np.array_equal(host(d[:k]), d2)
    assert bool((s != d).all()) and int(s.min()) >= 0 and int(d.max()) < n
    g = P.Graph(n, s, d)
    assert g.info["m"] == m  # every pair distinct
    s3, d3 = GEN.er(n, m, seed=2016, device=DEV)  # repeat call: the same list
    assert torch.equal(s, s3) and torch.equal(d, d3)


@pytest.mark.parametrize("n,k", [(2, 1), (3, 2), (17, 16), (1000, 3), (20_000, 1), (65_536, 16), (1_000_000, 8),
                                 (300, 255)])
@pytest.mark.parametrize("seed", [5, 2**63 + 11])
def test_ba_against_oracle(n, k, seed):
    print(f"[gen ba] n={n} k={k} seed={seed}", flush=True)
    s, d = GEN.ba(n, k, seed=seed, device=DEV)
    torch.cuda.synchronize()
    s2, d2 = oracle.ba(n, k, seed)
    assert np.array_equal(host(s), s2) and np.array_equal(host(d), d2)


def test_ba_large_properties_and_repeat():
    n, k = 1 << 22, 16
    s, d = GEN.ba(n, k, seed=22, device=DEV)
    torch.cuda.synchronize()
    es = k * (k + 1) // 2
    dv = d[es:].view(-1, k)
    v = torch.arange(k + 1, n, device=DEV, dtype=torch.int32)
    assert bool((s[es:].view(-1, k) == v[:, None]).all()) and bool((dv < v[:, None]).all())
    srt, _ = torch.sort(dv, dim=1)
    assert bool((srt[:, 1:] != srt[:, :-1]).all())  # k distinct targets per node
    m1 = 1 << 20
    s2, d2 = oracle.ba(m1 // k, k, 22)  # a smaller graph of the same seed is a prefix
    assert np.array_equal(host(d[:d2.size]), d2) and np.array_equal(host(s[:s2.size]), s2)
    g = P.Graph(n, s, d)
    assert g.info["m"] == s.numel()  # BA targets are distinct and earlier: no repeated pair
    s3, d3 = GEN.ba(n, k, seed=22, device=DEV)
    assert torch.equal(s, s3) and torch.equal(d, d3)


def test_generator_errors():
    L = N.lib()
    import ctypes
    b = ctypes.c_size_t()
    assert L.tricc_gen_er_workspace_size(10, 46, ctypes.byref(b)) == N.TRICC_EINVAL  # m > N = 45
    assert L.tricc_gen_er_workspace_size(-1, 0, ctypes.byref(b)) == N.TRICC_EINVAL
    assert L.tricc_gen_ba_edges(5, 5) == -1 and L.tricc_gen_ba_edges(5, 0) == -1 and L.tricc_gen_ba_edges(300, 256) == -1
    ws = torch.empty(256, dtype=torch.uint8, device=DEV)
    out = torch.empty(10, dtype=torch.int32, device=DEV)
    p = ctypes.c_void_p
    assert L.tricc_gen_er(100, 10, 1, p(out.data_ptr()), p(out.data_ptr()), p(ws.data_ptr()), 16, None) == \
        N.TRICC_ENOMEM
    with pytest.raises(ValueError):
        GEN.ba(4, 4, device=DEV)

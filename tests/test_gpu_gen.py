"""GPU parity of the device R-MAT generator (tricc_gen_rmat) against the
oracle's R-MAT of the same definition: edges compared bit-exactly over
scales, edge counts with ragged tails, noise levels, quadrant weights,
seeds and relabellings; the host input generator end to end; the full
benchmark size on sampled edges; repeat calls; and the argument errors."""
import numpy as np
import pytest
import torch

import oracle
import paper_1606_07550_amd as P
from paper_1606_07550_amd import _native as N
from paper_1606_07550_amd import inputs as I
from paper_1606_07550_amd.generators import rmat as gpu_rmat

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("scale,m", [(1, 1), (2, 255), (7, 256), (7, 257), (13, 100_003), (16, 1 << 20)])
@pytest.mark.parametrize("noise", [0.0, 0.1, 1.0])
def test_against_oracle(scale, m, noise):
    seed = 1000 * scale + m
    s, d = gpu_rmat(scale, m, noise=noise, seed=seed, device=DEV)
    torch.cuda.synchronize()
    s2, d2 = oracle.rmat(scale, m, noise=noise, seed=seed)
    assert np.array_equal(host(s), s2) and np.array_equal(host(d), d2)


@pytest.mark.parametrize("abcd", [(0.25, 0.25, 0.25, 0.25), (0.45, 0.15, 0.15, 0.25), (0.0, 1.0, 0.0, 0.0),
                                  (3.0, 1.0, 1.0, 0.5)])
@pytest.mark.parametrize("seed", [0, 2**64 - 1])
def test_weights_and_seeds(abcd, seed):
    s, d = gpu_rmat(11, 50_001, abcd=abcd, noise=0.3, seed=seed, device=DEV)
    s2, d2 = oracle.rmat(11, 50_001, abcd=abcd, noise=0.3, seed=seed)
    assert np.array_equal(host(s), s2) and np.array_equal(host(d), d2)


def test_relabelled_equals_host_input_generator():
    # the host generator's relabelled R-MAT, end to end, from the device
    for scale, seed in ((10, 3), (16, 16)):
        n, s, d = I.rmat(scale, 16, seed=seed)
        perm = torch.from_numpy(I.rmat_perm(scale, seed)).to(DEV)
        gs, gd = gpu_rmat(scale, seed=seed, perm=perm)
        assert np.array_equal(host(gs), s) and np.array_equal(host(gd), d)


def test_graph_from_device_edges():
    n, s, d = I.rmat(14, 16, seed=14)
    perm = torch.from_numpy(I.rmat_perm(14, 14)).to(DEV)
    gs, gd = gpu_rmat(14, seed=14, perm=perm)
    g = P.Graph(n, gs, gd)
    r = g.count()
    torch.cuda.synchronize()
    ref = oracle.count(n, s, d, order=1)
    assert np.array_equal(r["T"].cpu().numpy().view(np.uint64), ref["T"])
    assert int(r["total"].cpu().numpy().view(np.uint64)[0]) == ref["total"]


def test_repeat_calls_and_output_buffers():
    out = (torch.full((70_000,), -7, dtype=torch.int32, device=DEV),
           torch.full((70_000,), -7, dtype=torch.int32, device=DEV))
    a = gpu_rmat(12, 60_000, seed=9, out=out)
    first = (host(a[0]).copy(), host(a[1]).copy())
    s = torch.cuda.Stream()
    b = gpu_rmat(12, 60_000, seed=9, out=out, stream=s)
    s.synchronize()
    assert np.array_equal(first[0], host(b[0])) and np.array_equal(first[1], host(b[1]))
    assert (host(out[0])[60_000:] == -7).all()  # nothing past m is written


def test_zero_edges():
    s, d = gpu_rmat(5, 0, device=DEV)
    torch.cuda.synchronize()
    assert s.numel() == 0 and d.numel() == 0


def test_full_size_sampled():
    # R-MAT 24, edge factor 16 (268M pairs), relabelled: sampled edges
    # against the oracle one by one, every id in range
    scale, seed = 24, 24
    perm_h = I.rmat_perm(scale, seed)
    perm = torch.from_numpy(perm_h).to(DEV)
    s, d = gpu_rmat(scale, seed=seed, perm=perm)
    torch.cuda.synchronize()
    m = s.numel()
    assert m == 16 << scale
    assert int(s.min()) >= 0 and int(s.max()) < (1 << scale)
    assert int(d.min()) >= 0 and int(d.max()) < (1 << scale)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.integers(0, m, 200_000), [0, 1, 255, 256, m - 257, m - 1]]))
    ti = torch.from_numpy(idx).to(DEV)
    gs, gd = host(s[ti]), host(d[ti])
    s2, d2 = oracle.rmat(scale, idx=idx, seed=seed, perm=perm_h)
    assert np.array_equal(gs, s2) and np.array_equal(gd, d2)


@pytest.mark.parametrize("kw", [dict(scale=0), dict(scale=31), dict(m=-1), dict(abcd=(-0.1, 0.5, 0.3, 0.3)),
                                dict(abcd=(float("nan"), 0.5, 0.3, 0.3)), dict(abcd=(0.0, 0.0, 0.0, 0.0)),
                                dict(noise=1.5), dict(noise=-0.1)])
def test_bad_arguments(kw):
    args = dict(scale=5, m=10, abcd=(0.57, 0.19, 0.19, 0.05), noise=0.1)
    args.update(kw)
    out = (torch.empty(16, dtype=torch.int32, device=DEV), torch.empty(16, dtype=torch.int32, device=DEV))
    a, b, c, d = args["abcd"]
    rc = N.lib().tricc_gen_rmat(args["scale"], args["m"], a, b, c, d, args["noise"], 0, None,
                                out[0].data_ptr(), out[1].data_ptr(), None)
    assert rc == N.TRICC_EINVAL

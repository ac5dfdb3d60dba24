"""Graph generators on the device (argument marshalling only; the HIP
kernels of ``libtricc.so`` draw every edge)."""
import ctypes

import torch

from . import _native as N
from .graph import _ptr, _stream_ptr

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def rmat(scale, m=None, edge_factor=16, abcd=RMAT_ABCD, noise=0.1, seed=0, perm=None, device="cuda",
         out=None, stream=None):
    """R-MAT edge list on the device: (src, dst) int32 tensors of m =
    edge_factor * 2**scale pairs unless ``m`` is given (self loops and
    duplicates kept). ``perm`` (int32 device tensor of 2**scale ids)
    relabels both ends. Asynchronous on ``stream``."""
    m = edge_factor << scale if m is None else int(m)
    if perm is not None:
        if perm.dtype != torch.int32 or perm.numel() != 1 << scale or not perm.is_cuda:
            raise ValueError("perm must be an int32 device tensor of 2**scale ids")
        perm = perm.contiguous()
    if out is None:
        dev = perm.device if perm is not None else torch.device(device)
        out = (torch.empty(m, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev))
    src, dst = out
    if src.numel() < m or dst.numel() < m or src.dtype != torch.int32 or dst.dtype != torch.int32:
        raise ValueError("outputs must be int32 tensors of at least m elements")
    a, b, c, d = abcd
    with torch.cuda.device(src.device):
        rc = N.lib().tricc_gen_rmat(scale, m, a, b, c, d, noise, ctypes.c_uint64(seed & (2**64 - 1)),
                                    _ptr(perm), _ptr(src), _ptr(dst), _stream_ptr(stream))
    N.check(rc, "tricc_gen_rmat")
    return src[:m], dst[:m]


def _ws(nbytes, dev, workspace):
    if workspace is not None:
        if workspace.numel() < nbytes:
            raise ValueError(f"workspace of {workspace.numel()} bytes, {nbytes} needed")
        return workspace
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)


def er(n, m, seed=0, device="cuda", out=None, workspace=None, stream=None):
    """Erdos-Renyi G(n, m) on the device: (src, dst) int32 tensors of m
    distinct node pairs, no self loops (the first m distinct draws of a
    counter-based sequence of pair indices). Synchronises ``stream``."""
    m = int(m)
    need = ctypes.c_size_t()
    N.check(N.lib().tricc_gen_er_workspace_size(int(n), m, ctypes.byref(need)), "tricc_gen_er_workspace_size")
    dev = torch.device(device) if out is None else out[0].device
    if out is None:
        out = (torch.empty(m, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev))
    src, dst = out
    if src.numel() < m or dst.numel() < m or src.dtype != torch.int32 or dst.dtype != torch.int32:
        raise ValueError("outputs must be int32 tensors of at least m elements")
    ws = _ws(need.value, dev, workspace)
    with torch.cuda.device(dev):
        rc = N.lib().tricc_gen_er(int(n), m, ctypes.c_uint64(seed & (2**64 - 1)), _ptr(src), _ptr(dst), _ptr(ws),
                                  ws.numel(), _stream_ptr(stream))
    N.check(rc, "tricc_gen_er")
    return src[:m], dst[:m]


def ba_edges(n, k):
    return int(N.lib().tricc_gen_ba_edges(int(n), int(k)))


def ba(n, k, seed=0, device="cuda", out=None, workspace=None, stream=None):
    """Barabasi-Albert on the device: the clique on nodes 0..k, then k
    distinct earlier targets per node drawn in proportion to degree; (src,
    dst) int32 tensors of k(k+1)/2 + (n-k-1)k edges. Synchronises."""
    m = ba_edges(n, k)
    if m < 0:
        raise ValueError("Barabasi-Albert: need 1 <= k <= 255 and k < n < 2^31")
    need = ctypes.c_size_t()
    N.check(N.lib().tricc_gen_ba_workspace_size(int(n), int(k), ctypes.byref(need)), "tricc_gen_ba_workspace_size")
    dev = torch.device(device) if out is None else out[0].device
    if out is None:
        out = (torch.empty(m, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev))
    src, dst = out
    if src.numel() < m or dst.numel() < m or src.dtype != torch.int32 or dst.dtype != torch.int32:
        raise ValueError("outputs must be int32 tensors of at least m elements")
    ws = _ws(need.value, dev, workspace)
    with torch.cuda.device(dev):
        rc = N.lib().tricc_gen_ba(int(n), int(k), ctypes.c_uint64(seed & (2**64 - 1)), _ptr(src), _ptr(dst),
                                  _ptr(ws), ws.numel(), _stream_ptr(stream))
    N.check(rc, "tricc_gen_ba")
    return src[:m], dst[:m]

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

"""Python face of the batched path: many independent graphs packed back to
back, counted by one persistent launch captured in a hipGraph."""
import ctypes

import numpy as np
import torch

from . import _native as N
from .graph import _ptr, _stream_ptr


def default_batch_tuning():
    t = N.BatchTuning()
    N.check(N.lib().tricc_batch_default_tuning(ctypes.byref(t)), "tricc_batch_default_tuning")
    return t


def batch_workspace_size(num_graphs, total_nodes, total_pairs):
    b = ctypes.c_size_t()
    N.check(N.lib().tricc_batch_workspace_size(num_graphs, total_nodes, total_pairs, ctypes.byref(b)),
            "tricc_batch_workspace_size")
    return b.value


def _as_batch_tuning(t):
    if t is None:
        return None
    return N.BatchTuning.from_dict(t) if isinstance(t, dict) else t


class Batch:
    """``node_off`` / ``edge_off``: host int64 arrays of G+1 offsets;
    ``src`` / ``dst``: device int32 arrays of local ids. The build runs in the
    constructor (synchronises); :meth:`plan` binds outputs and captures the
    count; :meth:`run` is one graph launch."""

    def __init__(self, node_off, edge_off, src, dst, tuning=None, stream=None, workspace=None):
        node_off = np.ascontiguousarray(node_off, dtype=np.int64)
        edge_off = np.ascontiguousarray(edge_off, dtype=np.int64)
        if node_off.shape != edge_off.shape or node_off.ndim != 1 or node_off.size < 1:
            raise ValueError("node_off and edge_off must be 1-D arrays of G+1 offsets")
        if src.dtype != torch.int32 or dst.dtype != torch.int32 or not (src.is_cuda and dst.is_cuda):
            raise TypeError("src and dst must be int32 device tensors")
        self.G = node_off.size - 1
        self.n_total = int(node_off[-1])
        self.m_total = int(edge_off[-1])
        if src.numel() != self.m_total or dst.numel() != self.m_total:
            raise ValueError("edge arrays do not match edge_off[-1]")
        self.device = src.device
        self.node_off = node_off
        self.edge_off = edge_off
        need = batch_workspace_size(self.G, self.n_total, self.m_total)
        self.ws = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8, device=self.device)
        self._src, self._dst = src.contiguous(), dst.contiguous()
        self._h = ctypes.c_void_p()
        t = _as_batch_tuning(tuning)
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_batch_build(
                self.G, node_off.ctypes.data_as(ctypes.c_void_p), edge_off.ctypes.data_as(ctypes.c_void_p),
                _ptr(self._src), _ptr(self._dst), _ptr(self.ws), self.ws.numel(),
                ctypes.byref(t) if t is not None else None, _stream_ptr(stream), ctypes.byref(self._h))
        N.check(rc, "tricc_batch_build")
        self.out = None

    @classmethod
    def from_csr(cls, node_off, rowptr, col, assume_simple_sorted_symmetric=False, tuning=None, stream=None,
                 workspace=None):
        """A batch handed over as a packed CSR: ``node_off`` host int64[G+1];
        ``rowptr`` device int64[total nodes + 1] over ``col`` (device int32,
        local ids). Builds in the constructor (synchronises)."""
        node_off = np.ascontiguousarray(node_off, dtype=np.int64)
        if node_off.ndim != 1 or node_off.size < 1:
            raise ValueError("node_off must be a 1-D array of G+1 offsets")
        if rowptr.dtype != torch.int64 or col.dtype != torch.int32 or not (rowptr.is_cuda and col.is_cuda):
            raise TypeError("rowptr must be an int64 and col an int32 device tensor")
        self = cls.__new__(cls)
        self.G = node_off.size - 1
        self.n_total = int(node_off[-1])
        self.m_total = int(col.numel())
        if rowptr.numel() != self.n_total + 1:
            raise ValueError("rowptr must hold total nodes + 1 offsets")
        self.device = col.device
        self.node_off = node_off
        self.edge_off = None
        need = batch_workspace_size(self.G, self.n_total, self.m_total)
        self.ws = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8, device=self.device)
        self._src, self._dst = rowptr.contiguous(), col.contiguous()
        self._h = ctypes.c_void_p()
        t = _as_batch_tuning(tuning)
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_batch_build_csr(
                self.G, node_off.ctypes.data_as(ctypes.c_void_p), self.m_total, _ptr(self._src), _ptr(self._dst),
                int(bool(assume_simple_sorted_symmetric)), _ptr(self.ws), self.ws.numel(),
                ctypes.byref(t) if t is not None else None, _stream_ptr(stream), ctypes.byref(self._h))
        N.check(rc, "tricc_batch_build_csr")
        self.out = None
        return self

    @property
    def info(self):
        i = N.BatchInfo()
        N.check(N.lib().tricc_batch_info_get(self._h, ctypes.byref(i)), "tricc_batch_info_get")
        return i.as_dict()

    def plan(self, stream=None):
        dev = self.device
        self.out = {
            "T": torch.empty(max(self.n_total, 0), dtype=torch.int64, device=dev),
            "cc": torch.empty(max(self.n_total, 0), dtype=torch.float32, device=dev),
            "graph_tri": torch.empty(max(self.G, 0), dtype=torch.int64, device=dev),
            "graph_avg": torch.empty(max(self.G, 0), dtype=torch.float64, device=dev),
            "batch_tri": torch.zeros(1, dtype=torch.int64, device=dev),
        }
        o = self.out
        with torch.cuda.device(dev):
            rc = N.lib().tricc_batch_plan(self._h, _ptr(o["T"]), _ptr(o["cc"]), _ptr(o["graph_tri"]),
                                          _ptr(o["graph_avg"]), _ptr(o["batch_tri"]), _stream_ptr(stream))
        N.check(rc, "tricc_batch_plan")
        return o

    def graph_arrays(self):
        """Device views (slices of the workspace) of the union graph: deg
        int32[total nodes] (degrees in each member's simple graph) and doff
        int64[total nodes + 1] (its DAG offsets)."""
        h = N.lib().tricc_batch_graph(self._h)
        ptrs = [ctypes.c_void_p() for _ in range(5)]
        N.check(N.lib().tricc_graph_arrays(h, *[ctypes.byref(p) for p in ptrs]), "tricc_graph_arrays")
        base = self.ws.data_ptr()

        def view(p, dtype, count):
            off = p.value - base
            esz = torch.empty((), dtype=dtype).element_size()
            return self.ws[off:off + count * esz].view(dtype)

        return {"deg": view(ptrs[1], torch.int32, self.n_total), "doff": view(ptrs[3], torch.int64, self.n_total + 1)}

    def run(self, stream=None):
        N.check(N.lib().tricc_batch_run(self._h, _stream_ptr(stream)), "tricc_batch_run")
        return self.out

    def run_eager(self, stream=None):
        N.check(N.lib().tricc_batch_run_eager(self._h, _stream_ptr(stream)), "tricc_batch_run_eager")
        return self.out

    def retune(self, tuning, stream=None):
        t = _as_batch_tuning(tuning)
        N.check(N.lib().tricc_batch_retune(self._h, ctypes.byref(t), _stream_ptr(stream)), "tricc_batch_retune")

    def close(self):
        if self._h:
            N.lib().tricc_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

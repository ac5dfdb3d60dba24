"""Python face of the single-graph path: build a graph from an edge list held
in device memory, then count triangles and clustering coefficients.

PyTorch supplies the device memory (tensors) and the stream; all computation
runs in ``libtricc.so``.
"""
import ctypes

import torch

from . import _native as N


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def default_tuning():
    t = N.Tuning()
    N.check(N.lib().tricc_default_tuning(ctypes.byref(t)), "tricc_default_tuning")
    return t


def variant_capacity(v):
    return N.lib().tricc_variant_capacity(v)


def variant_count():
    return N.lib().tricc_variant_count()


def workspace_size(n, m_raw):
    b = ctypes.c_size_t()
    N.check(N.lib().tricc_graph_workspace_size(n, m_raw, ctypes.byref(b)), "tricc_graph_workspace_size")
    return b.value


def _as_tuning(tuning):
    if tuning is None:
        return None
    if isinstance(tuning, dict):
        return N.Tuning.from_dict(tuning)
    return tuning


class Graph:
    """A graph built on the GPU from ``n`` and int32 device edge arrays.

    Steps a1..a5 (validate, symmetrise, dedup, drop loops, sort rows, orient
    by (degree, id), bin) run in the constructor, which synchronises the
    stream. :meth:`count` runs the intersection kernels and the epilogue
    asynchronously."""

    def __init__(self, n, src, dst, tuning=None, stream=None, workspace=None):
        if src.dtype != torch.int32 or dst.dtype != torch.int32:
            raise TypeError("edge arrays must be int32")
        if not (src.is_cuda and dst.is_cuda):
            raise TypeError("edge arrays must be device tensors")
        if src.shape != dst.shape or src.dim() != 1:
            raise ValueError("src and dst must be 1-D of equal length")
        src = src.contiguous()
        dst = dst.contiguous()
        self.n = int(n)
        self.m_raw = int(src.numel())
        self.device = src.device
        need = workspace_size(self.n, self.m_raw)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        self.ws = workspace
        self._h = ctypes.c_void_p()
        t = _as_tuning(tuning)
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_build(self.n, self.m_raw, _ptr(src), _ptr(dst), _ptr(self.ws),
                                           self.ws.numel(), ctypes.byref(t) if t is not None else None,
                                           _stream_ptr(stream), ctypes.byref(self._h))
        N.check(rc, "tricc_graph_build")

    @classmethod
    def from_csr(cls, n, rowptr, col, assume_simple_sorted_symmetric=False, tuning=None, stream=None,
                 workspace=None):
        """A graph built from a device CSR: row v is col[rowptr[v]:rowptr[v+1]]
        (rowptr int64[n+1], col int32). With assume_simple_sorted_symmetric
        the rows are taken as they are (strictly ascending, no self loops,
        symmetric) and the sort is skipped; otherwise every entry is a pair
        (v, w) for the full build."""
        if rowptr.dtype != torch.int64 or col.dtype != torch.int32:
            raise TypeError("rowptr must be int64 and col int32")
        if not (rowptr.is_cuda and col.is_cuda):
            raise TypeError("CSR arrays must be device tensors")
        if rowptr.dim() != 1 or rowptr.numel() != int(n) + 1 or col.dim() != 1:
            raise ValueError("rowptr must hold n + 1 offsets and col must be 1-D")
        rowptr = rowptr.contiguous()
        col = col.contiguous()
        self = cls.__new__(cls)
        self.n = int(n)
        self.m_raw = int(col.numel())
        self.device = rowptr.device
        need = workspace_size(self.n, self.m_raw)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        self.ws = workspace
        self._h = ctypes.c_void_p()
        t = _as_tuning(tuning)
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_from_csr(self.n, self.m_raw, _ptr(rowptr), _ptr(col),
                                              1 if assume_simple_sorted_symmetric else 0, _ptr(self.ws),
                                              self.ws.numel(), ctypes.byref(t) if t is not None else None,
                                              _stream_ptr(stream), ctypes.byref(self._h))
        N.check(rc, "tricc_graph_from_csr")
        return self

    @property
    def info(self):
        i = N.GraphInfo()
        N.check(N.lib().tricc_graph_info_get(self._h, ctypes.byref(i)), "tricc_graph_info_get")
        return i.as_dict()

    def stats(self, stream=None):
        """Computes the algorithmic sizes of the intersection work (list_elems,
        bin_list_elems, bin_edges of :attr:`info`); synchronises."""
        N.check(N.lib().tricc_graph_stats(self._h, _stream_ptr(stream)), "tricc_graph_stats")
        return self.info

    def retune(self, tuning, stream=None):
        t = _as_tuning(tuning)
        N.check(N.lib().tricc_graph_retune(self._h, ctypes.byref(t), _stream_ptr(stream)), "tricc_graph_retune")

    def count(self, out=None, stream=None):
        """Returns dict(T=uint64[n] as int64 tensor, cc=float32[n],
        total=uint64[1] as int64 tensor, avg=float64[1]), on the device."""
        n = self.n
        if out is None:
            out = {
                "T": torch.empty(max(n, 0), dtype=torch.int64, device=self.device),
                "cc": torch.empty(max(n, 0), dtype=torch.float32, device=self.device),
                "total": torch.empty(1, dtype=torch.int64, device=self.device),
                "avg": torch.empty(1, dtype=torch.float64, device=self.device),
            }
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_count(self._h, _ptr(out["T"]), _ptr(out["cc"]), _ptr(out["total"]),
                                     _ptr(out["avg"]), _stream_ptr(stream))
        N.check(rc, "tricc_count")
        return out

    def count_check(self, stream=None):
        """(total, sum of T(v)) of the last count, as the device computed them
        (synchronises): the total comes from the intersection kernels' own
        counters, the sum from the epilogue."""
        t, s = ctypes.c_uint64(), ctypes.c_uint64()
        N.check(N.lib().tricc_count_check(self._h, ctypes.byref(t), ctypes.byref(s), _stream_ptr(stream)),
                "tricc_count_check")
        return int(t.value), int(s.value)

    def has_edges(self, u, v, out=None, stream=None):
        """Edge-existence tests: u, v int32 device tensors of one shape;
        returns uint8 (1 edge, 0 no edge, 0xFF an id outside [0, n))."""
        if u.dtype != torch.int32 or v.dtype != torch.int32 or u.shape != v.shape:
            raise ValueError("u and v must be int32 tensors of one shape")
        u, v = u.contiguous(), v.contiguous()
        if out is None:
            out = torch.empty(u.shape, dtype=torch.uint8, device=u.device)
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_has_edges(self._h, u.numel(), _ptr(u), _ptr(v), _ptr(out), _stream_ptr(stream))
        N.check(rc, "tricc_graph_has_edges")
        return out

    def core(self, k_stop=-1, out=None, stream=None):
        """Core numbers: (int32 tensor[n], largest value). k_stop >= 0 gives
        min(core number, k_stop), so the k_stop-core is where it equals
        k_stop. Synchronises the stream."""
        n = self.n
        need = ctypes.c_size_t()
        N.check(N.lib().tricc_core_workspace_size(n, ctypes.byref(need)), "tricc_core_workspace_size")
        ws = torch.empty(need.value, dtype=torch.uint8, device=self.device)
        if out is None:
            out = torch.empty(max(n, 0), dtype=torch.int32, device=self.device)
        mx = ctypes.c_int32()
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_core(self._h, int(k_stop), _ptr(out) if n > 0 else None, _ptr(ws),
                                          need.value, ctypes.byref(mx), _stream_ptr(stream))
        N.check(rc, "tricc_graph_core")
        return out, int(mx.value)

    def degeneracy(self, stream=None):
        """Degeneracy ordering: (order int32[n], core int32[n], degeneracy),
        order[v] = the peeling round that removed v. Synchronises."""
        n = self.n
        need = ctypes.c_size_t()
        N.check(N.lib().tricc_core_workspace_size(n, ctypes.byref(need)), "tricc_core_workspace_size")
        ws = torch.empty(need.value, dtype=torch.uint8, device=self.device)
        order = torch.empty(max(n, 0), dtype=torch.int32, device=self.device)
        core = torch.empty(max(n, 0), dtype=torch.int32, device=self.device)
        mx = ctypes.c_int32()
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_degeneracy(self._h, _ptr(order) if n > 0 else None,
                                                _ptr(core) if n > 0 else None, _ptr(ws), need.value,
                                                ctypes.byref(mx), _stream_ptr(stream))
        N.check(rc, "tricc_graph_degeneracy")
        return order, core, int(mx.value)

    def reorient(self, key=None, stream=None):
        """Orients the DAG by (key[v], v) (an int32 device tensor of n values
        >= 0), or by degree when key is None, and re-bins. Synchronises."""
        if key is not None:
            if key.dtype != torch.int32 or not key.is_cuda or key.numel() != self.n:
                raise TypeError("key must be an int32 device tensor of n values")
            key = key.contiguous()
        self._key = key  # kept alive for the call
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_reorient(self._h, _ptr(key) if key is not None and self.n > 0 else None,
                                              _stream_ptr(stream))
        N.check(rc, "tricc_graph_reorient")

    def orient_degeneracy(self, stream=None):
        """Re-orients by the degeneracy ordering; returns its degeneracy."""
        order, _, dg = self.degeneracy(stream)
        self.reorient(order, stream)
        return dg

    def count_k5(self, out=None, stream=None):
        """Number of 5-cliques: uint64[1] (as an int64 tensor) on the device."""
        if out is None:
            out = torch.empty(1, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_count_k5(self._h, _ptr(out), _stream_ptr(stream))
        N.check(rc, "tricc_graph_count_k5")
        return out

    def count_k4(self, out=None, stream=None):
        """Number of 4-cliques: uint64[1] (as an int64 tensor) on the device.
        Asynchronous. Raises TriccError (TRICC_EOVERFLOW) when some out-degree
        of the degree-ordered DAG exceeds 4,096."""
        if out is None:
            out = torch.empty(1, dtype=torch.int64, device=self.device)
        with torch.cuda.device(self.device):
            rc = N.lib().tricc_graph_count_k4(self._h, _ptr(out), _stream_ptr(stream))
        N.check(rc, "tricc_graph_count_k4")
        return out

    def arrays(self):
        """Device views (slices of the workspace) of the simple graph and DAG:
        off[n+1] int64, deg[n] int32, adj int32, doff[n+1] int64, dcol[m] int32."""
        ptrs = [ctypes.c_void_p() for _ in range(5)]
        N.check(N.lib().tricc_graph_arrays(self._h, *[ctypes.byref(p) for p in ptrs]), "tricc_graph_arrays")
        base = self.ws.data_ptr()
        n = self.n
        info = self.info

        def view(p, dtype, count):
            off = p.value - base
            esz = torch.empty((), dtype=dtype).element_size()
            return self.ws[off:off + count * esz].view(dtype)

        return {
            "off": view(ptrs[0], torch.int64, n + 1),
            "deg": view(ptrs[1], torch.int32, n),
            "adj": view(ptrs[2], torch.int32, 2 * self.m_raw),
            "doff": view(ptrs[3], torch.int64, n + 1),
            "dcol": view(ptrs[4], torch.int32, info["m"]),
        }

    def close(self):
        if self._h:
            N.lib().tricc_graph_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def count(n, src, dst, tuning=None, stream=None):
    """One pass of the whole single-graph path: build + count."""
    g = Graph(n, src, dst, tuning=tuning, stream=stream)
    out = g.count(stream=stream)
    out["info"] = g.info
    out["graph"] = g
    return out

"""CPU oracle: exact triangle counts, clustering coefficients, edge tests,
core numbers, 4- and 5-clique counts, R-MAT, G(n, m) and Barabasi-Albert edges.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package. The product path never does, and it
shares no code with the GPU path: the arithmetic lives in the plain C file
``tricc_oracle.c`` (node iterator over sorted adjacency lists, FP64 clustering
coefficients; the edge-existence test as a search in the sorted edge set),
built by ``build.py`` into ``liboracle.so``.

The definitions it follows are stated at the top of ``tricc_oracle.c``: the
paper names node clustering coefficient and triangle counting among SNAP's
triadic-closure methods (Section 4, table of analytics methods) and keeps
sorted adjacency vectors per node (Section 5.1), without giving formulas.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.oracle_count.argtypes = [i64, i64, P, P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P]
        L.oracle_count.restype = ctypes.c_int
        L.oracle_induced.argtypes = [i64, i64, P, P, i64, P, ctypes.c_int, P, P, P, P, P]
        L.oracle_induced.restype = ctypes.c_int
        L.oracle_sampled.argtypes = [i64, i64, P, P, i64, P, P, P]
        L.oracle_sampled.restype = ctypes.c_int
        L.oracle_has_edges.argtypes = [i64, i64, P, P, i64, P, P, P]
        L.oracle_has_edges.restype = ctypes.c_int
        L.oracle_core.argtypes = [i64, i64, P, P, ctypes.c_int32, P]
        L.oracle_core.restype = ctypes.c_int
        L.oracle_k4.argtypes = [i64, i64, P, P, ctypes.c_int, ctypes.c_int, P]
        L.oracle_k4.restype = ctypes.c_int
        L.oracle_k5.argtypes = [i64, i64, P, P, ctypes.c_int, ctypes.c_int, P]
        L.oracle_k5.restype = ctypes.c_int
        L.oracle_splitmix64.argtypes = [ctypes.c_uint64, i64, P]
        L.oracle_splitmix64.restype = ctypes.c_int
        d = ctypes.c_double
        L.oracle_rmat.argtypes = [ctypes.c_int, d, d, d, d, d, ctypes.c_uint64, i64, P, P, P, P]
        L.oracle_rmat.restype = ctypes.c_int
        d_ = ctypes.c_double
        L.oracle_count_timed.argtypes = [i64, i64, P, P, ctypes.c_int, ctypes.c_int, i64, i64, i64, P, P, P, P, P, P]
        L.oracle_count_timed.restype = ctypes.c_int
        L.oracle_er.argtypes = [i64, i64, ctypes.c_uint64, P, P]
        L.oracle_er.restype = ctypes.c_int
        L.oracle_ba.argtypes = [i64, ctypes.c_int32, ctypes.c_uint64, P, P]
        L.oracle_ba.restype = ctypes.c_int
        L.oracle_wtime.argtypes = []
        L.oracle_wtime.restype = ctypes.c_double
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    pass


def count(n, src, dst, order=0, threads=0):
    """Whole-graph result: dict with T (uint64[n]), cc (float64[n]),
    deg (int64[n]), total (int), avg (float), m (undirected simple edges).
    ``order`` 0 ranks nodes by id, 1 by (degree, id)."""
    src, dst = _i32(src), _i32(dst)
    assert src.shape == dst.shape
    T = np.zeros(n, np.uint64)
    cc = np.zeros(n, np.float64)
    deg = np.zeros(n, np.int64)
    total = ctypes.c_uint64()
    avg = ctypes.c_double()
    m = ctypes.c_int64()
    rc = lib().oracle_count(n, src.size, _ptr(src), _ptr(dst), order, threads, _ptr(T), _ptr(cc),
                            _ptr(deg), ctypes.byref(total), ctypes.byref(avg), ctypes.byref(m))
    if rc:
        raise OracleError(f"oracle_count failed ({rc})")
    return dict(T=T, cc=cc, deg=deg, total=int(total.value), avg=float(avg.value), m=int(m.value))


def count_timed(n, src, dst, order=1, threads=0, stride=1, offset=0, stride1=0):
    """Oracle timing on a node sample: dict(build_s, count_s, tri, count1_s,
    tri1, m); tri = triangles whose lowest-ranked vertex v has v % stride ==
    offset (threads threads); with stride1 > 0 also tri1 / count1_s for v %
    stride1 == offset on one thread, on the same build."""
    src, dst = _i32(src), _i32(dst)
    tri, tri1, m = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int64()
    b, c, c1 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib().oracle_count_timed(n, src.size, _ptr(src), _ptr(dst), order, threads, stride, offset, stride1,
                                  ctypes.byref(tri), ctypes.byref(tri1), ctypes.byref(m), ctypes.byref(b),
                                  ctypes.byref(c), ctypes.byref(c1))
    if rc:
        raise OracleError(f"oracle_count_timed failed ({rc})")
    return dict(build_s=b.value, count_s=c.value, tri=int(tri.value), count1_s=c1.value, tri1=int(tri1.value),
                m=int(m.value))


def induced(n, src, dst, nodes, threads=0):
    """Result on the induced subgraph G[S], indexed by position in ``nodes``."""
    src, dst, S = _i32(src), _i32(dst), _i32(nodes)
    k = S.size
    T = np.zeros(k, np.uint64)
    cc = np.zeros(k, np.float64)
    total = ctypes.c_uint64()
    avg = ctypes.c_double()
    m = ctypes.c_int64()
    rc = lib().oracle_induced(n, src.size, _ptr(src), _ptr(dst), k, _ptr(S), threads, _ptr(T), _ptr(cc),
                              ctypes.byref(total), ctypes.byref(avg), ctypes.byref(m))
    if rc:
        raise OracleError(f"oracle_induced failed ({rc})")
    return dict(T=T, cc=cc, total=int(total.value), avg=float(avg.value), m=int(m.value))


def sampled(n, src, dst, samples):
    """T(s) and d(s) for distinct sampled nodes, from the raw edge list."""
    src, dst, S = _i32(src), _i32(dst), _i32(samples)
    T = np.zeros(S.size, np.uint64)
    deg = np.zeros(S.size, np.int64)
    rc = lib().oracle_sampled(n, src.size, _ptr(src), _ptr(dst), S.size, _ptr(S), _ptr(T), _ptr(deg))
    if rc:
        raise OracleError(f"oracle_sampled failed ({rc})")
    return dict(T=T, deg=deg)


def has_edges(n, src, dst, qu, qv):
    """uint8 per query pair: 1 edge, 0 no edge (self pairs included), 0xFF an
    id outside [0, n)."""
    src, dst, qu, qv = _i32(src), _i32(dst), _i32(qu), _i32(qv)
    assert qu.shape == qv.shape
    out = np.zeros(qu.size, np.uint8)
    rc = lib().oracle_has_edges(n, src.size, _ptr(src), _ptr(dst), qu.size, _ptr(qu), _ptr(qv), _ptr(out))
    if rc:
        raise OracleError(f"oracle_has_edges failed ({rc})")
    return out


def core(n, src, dst, k_stop=-1):
    """int32 core number of every node (k_stop >= 0: min(core, k_stop))."""
    src, dst = _i32(src), _i32(dst)
    out = np.zeros(n, np.int32)
    rc = lib().oracle_core(n, src.size, _ptr(src), _ptr(dst), k_stop, _ptr(out))
    if rc:
        raise OracleError(f"oracle_core failed ({rc})")
    return out


def k4(n, src, dst, order=0, threads=0):
    """Number of 4-cliques of the simple graph."""
    src, dst = _i32(src), _i32(dst)
    total = ctypes.c_uint64()
    rc = lib().oracle_k4(n, src.size, _ptr(src), _ptr(dst), order, threads, ctypes.byref(total))
    if rc:
        raise OracleError(f"oracle_k4 failed ({rc})")
    return int(total.value)


def k5(n, src, dst, order=0, threads=0):
    """Number of 5-cliques of the simple graph."""
    src, dst = _i32(src), _i32(dst)
    total = ctypes.c_uint64()
    rc = lib().oracle_k5(n, src.size, _ptr(src), _ptr(dst), order, threads, ctypes.byref(total))
    if rc:
        raise OracleError(f"oracle_k5 failed ({rc})")
    return int(total.value)


def splitmix64(state, count):
    """The first ``count`` SplitMix64 outputs from ``state`` (uint64 array)."""
    out = np.zeros(count, np.uint64)
    lib().oracle_splitmix64(state, count, _ptr(out))
    return out


def rmat(scale, m=None, abcd=(0.57, 0.19, 0.19, 0.05), noise=0.1, seed=0, idx=None, perm=None):
    """R-MAT edges (src, dst int32) of the GPU generator's definition: edges
    0..m-1, or the edges numbered in ``idx``; ``perm`` relabels both ends."""
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        k = idx.size
    else:
        k = int(m)
    if perm is not None:
        perm = _i32(perm)
        assert perm.size == 1 << scale
    src = np.zeros(k, np.int32)
    dst = np.zeros(k, np.int32)
    a, b, c, d = abcd
    rc = lib().oracle_rmat(scale, a, b, c, d, noise, seed, k, _ptr(idx) if idx is not None else None,
                           _ptr(perm) if perm is not None else None, _ptr(src), _ptr(dst))
    if rc:
        raise OracleError(f"oracle_rmat failed ({rc})")
    return src, dst


def er(n, m, seed):
    """G(n, m) edges (src, dst int32[m]) of the GPU generator's definition."""
    src = np.zeros(m, np.int32)
    dst = np.zeros(m, np.int32)
    rc = lib().oracle_er(n, m, seed, _ptr(src), _ptr(dst))
    if rc:
        raise OracleError(f"oracle_er failed ({rc})")
    return src, dst


def ba_edges(n, k):
    return k * (k + 1) // 2 + (n - k - 1) * k


def ba(n, k, seed):
    """Barabasi-Albert edges (src, dst int32) of the GPU generator's
    definition: the seed clique on 0..k, then k distinct targets per node."""
    if not (1 <= k <= 255 and k < n):
        raise OracleError("oracle_ba: need 1 <= k <= 255 and k < n")
    m = ba_edges(n, k)
    src = np.zeros(m, np.int32)
    dst = np.zeros(m, np.int32)
    rc = lib().oracle_ba(n, k, seed, _ptr(src), _ptr(dst))
    if rc:
        raise OracleError(f"oracle_ba failed ({rc})")
    return src, dst


def wtime():
    return lib().oracle_wtime()

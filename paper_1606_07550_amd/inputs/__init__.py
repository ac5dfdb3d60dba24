"""Seeded synthetic inputs: edge lists and query node sets.

This module holds input generation only, and none of the triangle or
clustering-coefficient arithmetic; both the GPU path and the CPU oracle are
fed from it. The heavy generators (R-MAT, G(n,m), Barabasi-Albert, batches,
BFS balls) are C++ in ``graphgen.cpp``; the small fixture families with
known triangle counts are plain numpy in ``fixtures.py``.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtricc_gen.so")
_L = None

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(verbose=False):
    cmd = ["g++", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c++17",
           os.path.join(HERE, "graphgen.cpp"), "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P, i64, u64, f64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
        L.gen_er.argtypes = [i64, i64, u64, P, P]
        L.gen_rmat.argtypes = [i32, i64, f64, f64, f64, f64, f64, u64, i32, i32, P, P]
        L.gen_rmat_perm.argtypes = [i32, u64, P]
        L.gen_ba_edges.argtypes = [i64, i64]
        L.gen_ba_edges.restype = i64
        L.gen_ba.argtypes = [i64, i64, u64, P, P]
        L.gen_batch_sizes.argtypes = [i64, u64, i64, i64, P, P, P, P]
        L.gen_batch_fill.argtypes = [i64, u64, i64, i64, P, i32, P, P]
        L.gen_query_sizes.argtypes = [i64, u64, i64, i64, P]
        L.gen_bfs_queries.argtypes = [i64, i64, P, P, i64, u64, P, P, i32, P, P, P]
        _L = L
    return _L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed ({rc})")


def er(n, m, seed):
    """G(n, m): m distinct pairs, no loops, random orientation."""
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    _check(_lib().gen_er(n, m, seed, _p(src), _p(dst)), "gen_er")
    return src, dst


def rmat(scale, edge_factor=16, seed=0, abcd=RMAT_ABCD, noise=0.1, permute=True, threads=0, m=None):
    """R-MAT edge list with 2**scale nodes and edge_factor * 2**scale pairs
    (loops and duplicates kept). Returns (n, src, dst)."""
    n = 1 << scale
    m = edge_factor * n if m is None else m
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    a, b, c, d = abcd
    _check(_lib().gen_rmat(scale, m, a, b, c, d, noise, seed, int(bool(permute)), threads, _p(src), _p(dst)),
           "gen_rmat")
    return n, src, dst


def rmat_perm(scale, seed=0):
    """The node relabelling rmat(..., permute=True) applies: int32 array,
    perm[old id] = new id over the 2**scale ids."""
    perm = np.empty(1 << scale, np.int32)
    _check(_lib().gen_rmat_perm(scale, seed, _p(perm)), "gen_rmat_perm")
    return perm


def ba(n, k, seed):
    """Barabasi-Albert graph on n nodes attaching k edges per new node."""
    m = _lib().gen_ba_edges(n, k)
    if m < 0:
        raise ValueError("need k >= 1 and n >= k + 1")
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    _check(_lib().gen_ba(n, k, seed, _p(src), _p(dst)), "gen_ba")
    return src, dst


def batch(G, master_seed, nmin=64, nmax=65536, threads=0):
    """A batch of G mixed BA / ER graphs. Local node ids; graph g owns edges
    [edge_off[g], edge_off[g+1]) and nodes [node_off[g], node_off[g+1])."""
    n = np.empty(G, np.int64)
    m = np.empty(G, np.int64)
    fam = np.empty(G, np.int32)
    par = np.empty(G, np.float64)
    _check(_lib().gen_batch_sizes(G, master_seed, nmin, nmax, _p(n), _p(m), _p(fam), _p(par)), "gen_batch_sizes")
    edge_off = np.zeros(G + 1, np.int64)
    np.cumsum(m, out=edge_off[1:])
    node_off = np.zeros(G + 1, np.int64)
    np.cumsum(n, out=node_off[1:])
    src = np.empty(int(edge_off[-1]), np.int32)
    dst = np.empty(int(edge_off[-1]), np.int32)
    _check(_lib().gen_batch_fill(G, master_seed, nmin, nmax, _p(edge_off), threads, _p(src), _p(dst)),
           "gen_batch_fill")
    return dict(n=n, m=m, family=fam, param=par, node_off=node_off, edge_off=edge_off, src=src, dst=dst)


def query_sizes(Q, seed, kmin=16, kmax=100_000):
    k = np.empty(Q, np.int64)
    _check(_lib().gen_query_sizes(Q, seed, kmin, kmax, _p(k)), "gen_query_sizes")
    return k


def bfs_queries(n, src, dst, Q, seed, kmin=16, kmax=100_000, threads=0):
    """Q BFS balls. Returns (offsets[Q+1], nodes, seeds): ball q is
    nodes[offsets[q]:offsets[q+1]] (its size may be below the requested one
    when the component is smaller)."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    k_req = query_sizes(Q, seed, kmin, kmax)
    q_off = np.zeros(Q + 1, np.int64)
    np.cumsum(k_req, out=q_off[1:])
    buf = np.empty(int(q_off[-1]), np.int32)
    k_act = np.empty(Q, np.int64)
    seeds = np.empty(Q, np.int32)
    _check(_lib().gen_bfs_queries(n, src.size, _p(src), _p(dst), Q, seed, _p(k_req), _p(q_off), threads,
                                  _p(buf), _p(k_act), _p(seeds)), "gen_bfs_queries")
    off = np.zeros(Q + 1, np.int64)
    np.cumsum(k_act, out=off[1:])
    nodes = np.empty(int(off[-1]), np.int32)
    for q in range(Q):
        nodes[off[q]:off[q + 1]] = buf[q_off[q]:q_off[q] + k_act[q]]
    return off, nodes, seeds


def poisson_arrivals(Q, rate, seed):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=Q))


def log_uniform_int(rng, lo, hi, size=None):
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)

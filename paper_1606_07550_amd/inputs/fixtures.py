"""Small deterministic graph families with known triangle structure.

The paper's generator table lists complete graphs, circles, grids, stars and
trees as regular families and Watts-Strogatz among the random ones; wheels,
windmills and complete bipartite graphs are added because their counts have
simple closed forms. Each function returns (n, src, dst) as int32 numpy
arrays; none holds any triangle arithmetic.
"""
import numpy as np


def _pack(n, pairs):
    a = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    return n, a[:, 0].astype(np.int32), a[:, 1].astype(np.int32)


def complete(n):
    return _pack(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def ring(n):
    return _pack(n, [(i, (i + 1) % n) for i in range(n)] if n >= 3 else [(0, 1)] if n == 2 else [])


def path(n):
    return _pack(n, [(i, i + 1) for i in range(n - 1)])


def star(leaves):
    return _pack(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def random_tree(n, seed):
    rng = np.random.default_rng(seed)
    return _pack(n, [(int(rng.integers(0, i)), i) for i in range(1, n)])


def grid(r, c):
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return _pack(r * c, pairs)


def complete_bipartite(a, b):
    return _pack(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def random_bipartite(a, b, p, seed):
    rng = np.random.default_rng(seed)
    mask = rng.random((a, b)) < p
    ii, jj = np.nonzero(mask)
    return _pack(a + b, list(zip(ii.tolist(), (jj + a).tolist())))


def wheel(r):
    """Hub 0 joined to every node of the rim cycle 1..r."""
    pairs = [(0, i) for i in range(1, r + 1)]
    pairs += [(i, i % r + 1) for i in range(1, r + 1)]
    return _pack(r + 1, pairs)


def windmill(k):
    """k triangles sharing the centre 0: (0, 2i+1, 2i+2)."""
    pairs = []
    for i in range(k):
        a, b = 2 * i + 1, 2 * i + 2
        pairs += [(0, a), (0, b), (a, b)]
    return _pack(2 * k + 1, pairs)


def ring_lattice(n, K):
    """Watts-Strogatz ring lattice (rewiring probability 0): node i joined to
    the K/2 nearest nodes on each side."""
    assert K % 2 == 0
    return _pack(n, [(i, (i + s) % n) for i in range(n) for s in range(1, K // 2 + 1)])


def disjoint_union(*graphs):
    n0 = 0
    S, D = [], []
    for n, s, d in graphs:
        S.append(s.astype(np.int64) + n0)
        D.append(d.astype(np.int64) + n0)
        n0 += n
    if not S:
        return 0, np.zeros(0, np.int32), np.zeros(0, np.int32)
    return n0, np.concatenate(S).astype(np.int32), np.concatenate(D).astype(np.int32)


def messy(n, src, dst, seed, dup_frac=0.3, loops=5):
    """Same simple graph, noisier input: shuffled pairs, some reversed, some
    repeated, and a few self loops added."""
    rng = np.random.default_rng(seed)
    s = src.astype(np.int64)
    d = dst.astype(np.int64)
    k = int(len(s) * dup_frac)
    if len(s):
        idx = rng.integers(0, len(s), size=k)
        s = np.concatenate([s, d[idx]])
        d = np.concatenate([d, s[idx]])
    if n > 0 and loops:
        lv = rng.integers(0, n, size=loops)
        s = np.concatenate([s, lv])
        d = np.concatenate([d, lv])
    flip = rng.random(len(s)) < 0.5
    s, d = np.where(flip, d, s), np.where(flip, s, d)
    perm = rng.permutation(len(s))
    return n, s[perm].astype(np.int32), d[perm].astype(np.int32)


def relabel(n, src, dst, seed):
    """Random relabelling of node ids; returns (n, src, dst, perm) with new id
    perm[old]."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).astype(np.int64)
    return n, perm[src].astype(np.int32), perm[dst].astype(np.int32), perm


def k4_core(core, centres, avg_deg, seed):
    """Centres 0..centres-1, pairwise adjacent and joined to every node of a
    core of `core` nodes that carries a seeded sparse random graph of average
    degree `avg_deg`; each core node also gets core + centres + 1 private
    leaves. Core nodes then outrank the centres in (degree, id) order, so a
    centre's out-list holds the whole core (plus the centres above it): its
    out-degree lands between `core` and `core + centres - 1`, in the range of
    a chosen 4-clique kernel, while its rows stay sparse."""
    rng = np.random.default_rng(seed)
    c0 = centres
    pairs = [(a, b) for a in range(centres) for b in range(a + 1, centres)]
    ci = np.repeat(np.arange(centres), core)
    cj = np.tile(np.arange(core), centres) + c0
    m_in = int(core * avg_deg // 2)
    ia = rng.integers(0, core, size=m_in) + c0
    ib = rng.integers(0, core, size=m_in) + c0
    L = core + centres + 1
    la = np.repeat(np.arange(core), L) + c0
    lb = np.arange(core * L) + c0 + core
    s = np.concatenate([np.asarray([p[0] for p in pairs], np.int64), ci, ia, la])
    d = np.concatenate([np.asarray([p[1] for p in pairs], np.int64), cj, ib, lb])
    return c0 + core + core * L, s.astype(np.int32), d.astype(np.int32)


# (core, centres, avg_deg, seed): the centres' out-degrees fall just above
# 1,024, inside (1,024, 2,048], (2,048, 4,096] and (4,096, 8,192]
K4_CORE_CASES = [(1030, 3, 240, 71), (1500, 4, 90, 72), (2100, 2, 60, 73), (3500, 3, 40, 74), (5000, 2, 40, 75)]

# the same construction for 5-cliques: centres' out-degrees in (512, 1,024]
# (the larger 5-clique kernel) with denser cores
K5_CORE_CASES = [(600, 4, 120, 81), (1000, 3, 200, 82)]

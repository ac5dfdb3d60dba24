// Seeded synthetic graph generators.
//
// This file holds input generation only: it draws edge lists and query node
// sets, and contains none of the triangle / clustering-coefficient arithmetic.
// Both the GPU path and the CPU oracle are fed from it.
//
// Random numbers come from the SplitMix64 output function (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), used
// either as a counter-based generator (draw(seed, stream, counter)) where the
// work is parallel, or stepped sequentially where it is not.
//
// Generators (the paper's generator table names each family):
//   * Erdos-Renyi G(n,m): a uniform m-subset of the n(n-1)/2 node pairs, by
//     Floyd's sampling (Bentley and Floyd, CACM 1987) over pair indices.
//   * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004) with per-edge, per-level
//     multiplicative noise on (a,b,c,d) and a seeded node-id permutation.
//   * Barabasi-Albert preferential attachment from a (k+1)-clique seed.
//   * a batch of mixed BA / ER graphs with log-uniform sizes.
//   * breadth-first-search balls around random seeds (query node sets).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Counter-based draw: independent 64-bit value for (seed, stream, counter).
inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return mix64(mix64(seed + kGolden * (stream + 1)) + kGolden * (ctr + 1));
}

inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// Uniform integer in [0, bound) by the multiply-high method (Lemire 2019);
// the bias is below bound / 2^64 and is ignored.
inline uint64_t below(uint64_t x, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)x * bound) >> 64);
}

struct SeqRng {  // sequential SplitMix64
  uint64_t s;
  explicit SeqRng(uint64_t seed) : s(seed) {}
  uint64_t next() { s += kGolden; return mix64(s); }
};

enum : uint64_t {
  kStreamRmat = 11, kStreamPerm = 12, kStreamEr = 13, kStreamErFlip = 14,
  kStreamBa = 15, kStreamBatch = 16, kStreamQuery = 17,
};

// Open-addressing set of uint64 keys (Floyd sampling); key ~0 marks empty.
struct U64Set {
  std::vector<uint64_t> slot;
  uint64_t mask;
  explicit U64Set(uint64_t want) {
    uint64_t cap = 16;
    while (cap < 2 * want + 16) cap <<= 1;
    slot.assign(cap, ~0ULL);
    mask = cap - 1;
  }
  bool insert(uint64_t k) {  // true if newly inserted
    uint64_t h = mix64(k) & mask;
    while (true) {
      uint64_t s = slot[h];
      if (s == ~0ULL) { slot[h] = k; return true; }
      if (s == k) return false;
      h = (h + 1) & mask;
    }
  }
};

// Pair index k -> (i, j), 0 <= i < j, k = j(j-1)/2 + i.
inline void unrank_pair(uint64_t k, uint64_t* i, uint64_t* j) {
  uint64_t jj = (uint64_t)((1.0 + std::sqrt(1.0 + 8.0 * (double)k)) * 0.5);
  while (jj > 1 && jj * (jj - 1) / 2 > k) --jj;
  while ((jj + 1) * jj / 2 <= k) ++jj;
  *j = jj;
  *i = k - jj * (jj - 1) / 2;
}

void er_fill(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
  const uint64_t N = (uint64_t)n * (uint64_t)(n - 1) / 2;
  U64Set set((uint64_t)m);
  SeqRng rng(draw(seed, kStreamEr, 0));
  int64_t out = 0;
  for (uint64_t j = N - (uint64_t)m; j < N; ++j) {
    uint64_t t = below(rng.next(), j + 1);
    uint64_t pick = set.insert(t) ? t : (set.insert(j), j);
    uint64_t a, b;
    unrank_pair(pick, &a, &b);
    // random orientation, so that consumers must symmetrise
    if (draw(seed, kStreamErFlip, (uint64_t)out) & 1) std::swap(a, b);
    src[out] = (int32_t)a;
    dst[out] = (int32_t)b;
    ++out;
  }
}

int64_t ba_edges(int64_t n, int64_t k) { return k * (k + 1) / 2 + (n - k - 1) * k; }

void ba_fill(int64_t n, int64_t k, uint64_t seed, int32_t* src, int32_t* dst) {
  const int64_t m = ba_edges(n, k);
  std::vector<int32_t> ends;
  ends.reserve(2 * m);
  int64_t out = 0;
  for (int64_t i = 0; i <= k; ++i)
    for (int64_t j = i + 1; j <= k; ++j) {
      src[out] = (int32_t)i; dst[out] = (int32_t)j; ++out;
      ends.push_back((int32_t)i); ends.push_back((int32_t)j);
    }
  SeqRng rng(draw(seed, kStreamBa, 0));
  std::vector<int32_t> tgt(k);
  for (int64_t t = k + 1; t < n; ++t) {
    int64_t got = 0;
    while (got < k) {
      int32_t c = ends[below(rng.next(), ends.size())];
      bool dup = false;
      for (int64_t q = 0; q < got; ++q) dup |= (tgt[q] == c);
      if (!dup) tgt[got++] = c;
    }
    for (int64_t q = 0; q < k; ++q) {
      src[out] = (int32_t)t; dst[out] = tgt[q]; ++out;
      ends.push_back((int32_t)t); ends.push_back(tgt[q]);
    }
  }
}

struct BatchSpec { int64_t n, m; int family, k; double dbar; };

BatchSpec batch_spec(uint64_t master, int64_t g, int64_t nmin, int64_t nmax) {
  const uint64_t s = mix64(master + kGolden * (uint64_t)(g + 1));
  BatchSpec b{};
  b.family = (int)(draw(s, kStreamBatch, 0) & 1);  // 0 = BA, 1 = ER
  const double lo = std::log((double)nmin), hi = std::log((double)nmax);
  b.n = (int64_t)std::llround(std::exp(lo + u01(draw(s, kStreamBatch, 1)) * (hi - lo)));
  if (b.n < nmin) b.n = nmin;
  if (b.n > nmax) b.n = nmax;
  if (b.family == 1) {
    b.dbar = 4.0 + 28.0 * u01(draw(s, kStreamBatch, 2));
    int64_t m = (int64_t)std::llround((double)b.n * b.dbar / 2.0);
    const int64_t full = b.n * (b.n - 1) / 2;
    b.m = m < full ? m : full;
    b.k = 0;
  } else {
    b.k = 2 + (int)below(draw(s, kStreamBatch, 3), 15);  // {2..16}
    if (b.k + 1 > b.n) b.k = (int)b.n - 1;
    b.m = ba_edges(b.n, b.k);
    b.dbar = 0.0;
  }
  return b;
}

}  // namespace

// Seeded uniform random permutation of [0, n) (Fisher-Yates, sequential).
void rmat_perm(int64_t n, uint64_t seed, int32_t* perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  SeqRng rng(draw(seed, kStreamPerm, 0));
  for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[below(rng.next(), (uint64_t)i + 1)]);
}

extern "C" {

// Erdos-Renyi G(n,m). Writes m edges (no loops, no duplicate pairs, random
// orientation). Returns 0, or -1 if m exceeds n(n-1)/2 or n < 0.
int gen_er(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 0 || m < 0) return -1;
  const uint64_t N = n < 2 ? 0 : (uint64_t)n * (uint64_t)(n - 1) / 2;
  if ((uint64_t)m > N) return -1;
  if (m == 0) return 0;
  er_fill(n, m, seed, src, dst);
  return 0;
}

// R-MAT with 2^scale nodes and `m` edges. At each of the `scale` levels the
// quadrant probabilities (a,b,c,d) are multiplied by independent factors
// uniform in [1-noise, 1+noise] (16-bit resolution), renormalised, and one
// quadrant is drawn: a=(0,0) b=(0,1) c=(1,0) d=(1,1) for (src bit, dst bit),
// most significant bit first. If `permute`, node ids are then relabelled by
// a seeded uniform random permutation (Fisher-Yates). Self loops and
// duplicates are kept: the consumer removes them.
int gen_rmat(int scale, int64_t m, double a, double b, double c, double d, double noise,
             uint64_t seed, int permute, int nthreads, int32_t* src, int32_t* dst) {
  if (scale < 1 || scale > 30 || m < 0) return -1;
  const int64_t n = (int64_t)1 << scale;
  const double base[4] = {a, b, c, d};
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      const uint64_t ctr = ((uint64_t)e * (uint64_t)scale + (uint64_t)l) * 2;
      const uint64_t r1 = draw(seed, kStreamRmat, ctr);
      double p[4], sum = 0.0;
      for (int q = 0; q < 4; ++q) {
        const double f = 1.0 + noise * (2.0 * (double)((r1 >> (16 * q)) & 0xFFFF) / 65535.0 - 1.0);
        p[q] = base[q] * f;
        sum += p[q];
      }
      const double x = u01(draw(seed, kStreamRmat, ctr + 1)) * sum;
      int q = 3;
      if (x < p[0]) q = 0;
      else if (x < p[0] + p[1]) q = 1;
      else if (x < p[0] + p[1] + p[2]) q = 2;
      u = (u << 1) | (uint32_t)(q >> 1);
      v = (v << 1) | (uint32_t)(q & 1);
    }
    src[e] = (int32_t)u;
    dst[e] = (int32_t)v;
  }
  if (permute) {
    std::vector<int32_t> perm(n);
    rmat_perm(n, seed, perm.data());
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t e = 0; e < m; ++e) {
      src[e] = perm[src[e]];
      dst[e] = perm[dst[e]];
    }
  }
  return 0;
}

// The node relabelling gen_rmat applies when `permute` is set: perm[old id]
// = new id, for the 2^scale ids.
int gen_rmat_perm(int scale, uint64_t seed, int32_t* perm) {
  if (scale < 1 || scale > 30) return -1;
  rmat_perm((int64_t)1 << scale, seed, perm);
  return 0;
}

// Number of edges gen_ba writes for (n, k).
int64_t gen_ba_edges(int64_t n, int64_t k) { return (k < 1 || n < k + 1) ? -1 : ba_edges(n, k); }

// Barabasi-Albert: seed clique on nodes 0..k, then each new node attaches to
// k distinct earlier nodes drawn with probability proportional to degree.
int gen_ba(int64_t n, int64_t k, uint64_t seed, int32_t* src, int32_t* dst) {
  if (k < 1 || n < k + 1) return -1;
  ba_fill(n, k, seed, src, dst);
  return 0;
}

// Batch of G graphs: per graph a fair coin picks BA (k uniform in {2..16})
// or ER (average degree uniform in [4,32], m = round(n*dbar/2) capped at
// n(n-1)/2); n is log-uniform in [nmin, nmax]. Per-graph seeds are the
// SplitMix64 output of master + golden*(g+1). Fills n_out[G], m_out[G],
// family[G] (0 BA, 1 ER) and param[G] (k for BA, dbar for ER).
int gen_batch_sizes(int64_t G, uint64_t master, int64_t nmin, int64_t nmax,
                    int64_t* n_out, int64_t* m_out, int32_t* family, double* param) {
  if (G < 0 || nmin < 3 || nmax < nmin) return -1;
  for (int64_t g = 0; g < G; ++g) {
    BatchSpec b = batch_spec(master, g, nmin, nmax);
    n_out[g] = b.n; m_out[g] = b.m; family[g] = b.family;
    param[g] = b.family ? b.dbar : (double)b.k;
  }
  return 0;
}

// Fills the edges of every graph of the batch, local ids in [0, n_g), graph g
// at [edge_off[g], edge_off[g+1]).
int gen_batch_fill(int64_t G, uint64_t master, int64_t nmin, int64_t nmax,
                   const int64_t* edge_off, int nthreads, int32_t* src, int32_t* dst) {
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : bad)
  for (int64_t g = 0; g < G; ++g) {
    BatchSpec b = batch_spec(master, g, nmin, nmax);
    if (edge_off[g + 1] - edge_off[g] != b.m) { bad |= 1; continue; }
    const uint64_t s = mix64(master + kGolden * (uint64_t)(g + 1));
    int32_t* S = src + edge_off[g];
    int32_t* D = dst + edge_off[g];
    if (b.family) { if (b.m) er_fill(b.n, b.m, s, S, D); }
    else ba_fill(b.n, b.k, s, S, D);
  }
  return bad ? -1 : 0;
}

// Requested query sizes: k_q = round(exp(U[ln kmin, ln kmax])).
int gen_query_sizes(int64_t Q, uint64_t seed, int64_t kmin, int64_t kmax, int64_t* k_req) {
  if (Q < 0 || kmin < 1 || kmax < kmin) return -1;
  const double lo = std::log((double)kmin), hi = std::log((double)kmax);
  for (int64_t q = 0; q < Q; ++q) {
    int64_t k = (int64_t)std::llround(std::exp(lo + u01(draw(seed, kStreamQuery, 2 * q)) * (hi - lo)));
    k_req[q] = k < kmin ? kmin : (k > kmax ? kmax : k);
  }
  return 0;
}

// Breadth-first-search balls. For query q a seed node is drawn uniformly
// among nodes with at least one neighbour (ignoring self loops); BFS visits
// neighbours in ascending id order and the ball is the first k_req[q]
// discovered nodes (seed included), or the whole component if smaller.
// Output: ball q at nodes[q_off[q] .. q_off[q] + k_act[q]), q_off[q] is the
// prefix sum of k_req (so the caller sizes `nodes` as sum(k_req)).
int gen_bfs_queries(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst,
                    int64_t Q, uint64_t seed, const int64_t* k_req, const int64_t* q_off,
                    int nthreads, int32_t* nodes, int64_t* k_act, int32_t* seeds_out) {
  if (n <= 0) return -1;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t e = 0; e < m_raw; ++e) {
    const int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) return -2;
    if (u == v) continue;
    ++off[u + 1];
    ++off[v + 1];
  }
  for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
  std::vector<int32_t> adj(off[n]);
  {
    std::vector<int64_t> cur(off.begin(), off.end() - 1);
    for (int64_t e = 0; e < m_raw; ++e) {
      const int32_t u = src[e], v = dst[e];
      if (u == v) continue;
      adj[cur[u]++] = v;
      adj[cur[v]++] = u;
    }
  }
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nthreads)
  for (int64_t i = 0; i < n; ++i) std::sort(adj.begin() + off[i], adj.begin() + off[i + 1]);
  std::vector<int32_t> nonisolated;
  for (int64_t i = 0; i < n; ++i)
    if (off[i + 1] > off[i]) nonisolated.push_back((int32_t)i);
  if (nonisolated.empty()) return -3;
#pragma omp parallel num_threads(nthreads)
  {
    std::vector<int64_t> stamp(n, -1);
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < Q; ++q) {
      const int32_t s = nonisolated[below(draw(seed, kStreamQuery, 2 * q + 1), nonisolated.size())];
      int32_t* out = nodes + q_off[q];
      const int64_t k = k_req[q];
      int64_t head = 0, tail = 0;
      out[tail++] = s;
      stamp[s] = q;
      while (head < tail && tail < k) {
        const int32_t x = out[head++];
        for (int64_t p = off[x]; p < off[x + 1] && tail < k; ++p) {
          const int32_t y = adj[p];
          if (stamp[y] != q) { stamp[y] = q; out[tail++] = y; }
        }
      }
      k_act[q] = tail;
      if (seeds_out) seeds_out[q] = s;
    }
  }
  return 0;
}

}  // extern "C"

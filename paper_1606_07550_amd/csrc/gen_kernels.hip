// R-MAT edge generator on the device (the paper's table of graph generators,
// Section 4, cites Chakrabarti, Zhan and Faloutsos, SDM 2004): the recursive
// quadrant choice with per-level noise on (a, b, c, d), one edge per lane.
//
// Random bits are counter-based: word(c) is the SplitMix64 output function
// (Steele, Lea and Flood, OOPSLA 2014) of S + gamma * c, with
// S = out(seed + 12 gamma) and gamma the 64-bit golden-ratio increment. Level
// l of edge e reads word(k + 1) (four 16-bit noise fields) and word(k + 2)
// (the uniform draw), k = 2 (e * scale + l), so every edge is independent of
// every other and of the launch shape.
#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kGenNT = 256;

__host__ __device__ __forceinline__ uint64_t sm64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t sm64_host(uint64_t z) { return sm64(z); }

// 2h / 65535, correctly rounded, for 0 <= h < 2^16: the product with the
// rounded reciprocal, corrected once by its exact FMA residual (Markstein's
// method). Over all 65,536 values of h this equals IEEE division; the
// product alone is one ulp off for 88 of them.
__device__ __forceinline__ double two_h_over_65535(uint64_t h) {
#pragma clang fp contract(off)
  constexpr double r = 1.0 / 65535.0;
  const double n = 2.0 * (double)h;
  const double q0 = n * r;
  return __builtin_fma(__builtin_fma(-q0, 65535.0, n), r, q0);
}

// Noisy weight of one quadrant: base * (1 + noise * (2 h / 65535 - 1)).
__device__ __forceinline__ double noisy(double base, double noise, uint64_t h) {
#pragma clang fp contract(off)
  return base * (1.0 + noise * (two_h_over_65535(h) - 1.0));
}

// Grid-stride over the edges. FP64 contraction is off: each product and sum
// is rounded on its own, in the order of the definition, so an edge is the
// same bit pattern whatever the compiler would fuse. perm (may be null)
// relabels both ends.
__global__ __launch_bounds__(kGenNT) void k_gen_rmat(int64_t m, int scale, double a, double b, double c,
                                                     double d, double noise, uint64_t seed,
                                                     const int32_t* __restrict__ perm,
                                                     int32_t* __restrict__ src, int32_t* __restrict__ dst) {
#pragma clang fp contract(off)
  const uint64_t S = sm64(seed + kGamma * 12u);
  const int64_t stride = (int64_t)gridDim.x * kGenNT;
  for (int64_t e = (int64_t)blockIdx.x * kGenNT + threadIdx.x; e < m; e += stride) {
    uint64_t t = S + kGamma * (2u * (uint64_t)e * (uint64_t)scale + 1u);  // S + gamma (k + 1), k of level 0
    uint32_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      const uint64_t w1 = sm64(t);
      const uint64_t w2 = sm64(t + kGamma);
      t += 2u * kGamma;
      const double p0 = noisy(a, noise, w1 & 0xFFFFu);
      const double p1 = noisy(b, noise, (w1 >> 16) & 0xFFFFu);
      const double p2 = noisy(c, noise, (w1 >> 32) & 0xFFFFu);
      const double p3 = noisy(d, noise, w1 >> 48);
      const double s01 = p0 + p1;
      const double s012 = s01 + p2;
      const double x = (double)(w2 >> 11) * 0x1.0p-53 * (s012 + p3);
      // first q with x below the prefix sum; the prefixes of non-negative
      // weights never decrease, so that is the number of prefixes <= x
      const uint32_t q = (uint32_t)(x >= p0) + (uint32_t)(x >= s01) + (uint32_t)(x >= s012);
      u = (u << 1) | (q >> 1);
      v = (v << 1) | (q & 1u);
    }
    if (perm) {
      src[e] = perm[u];
      dst[e] = perm[v];
    } else {
      src[e] = (int32_t)u;
      dst[e] = (int32_t)v;
    }
  }
}

// ---------------------------------------------------------------------------
// Erdos-Renyi G(n, m) (the paper's generator table, Section 4): a uniform
// m-subset of the N = n(n-1)/2 node pairs, drawn as the first m distinct
// values of the counter-based sequence x_k = floor(word(k + 1) N / 2^64),
// k = 0, 1, ... (word from S = out(seed + 13 gamma)); pair index t is
// unranked row by row, t = i n - i(i+1)/2 + (j - i - 1) for i < j, and the
// low bit of the word swaps the two ends. Rejecting repeats in draw order is
// the sequential definition; here every draw records itself in a hash table
// keyed by its value with the smallest draw index (atomic min), a draw is
// new when it holds that index, and an exclusive scan of the new-draw flags
// gives each new value its edge index.

constexpr uint64_t kErEmpty = ~0ull;
constexpr uint32_t kErNoIdx = 0xFFFFFFFFu;

__device__ __forceinline__ uint64_t er_word(uint64_t S, uint64_t k) { return sm64(S + kGamma * (k + 1u)); }

__device__ __forceinline__ uint64_t er_slot(uint64_t x, uint64_t mask) { return sm64(x ^ 0x5851F42D4C957F2Dull) & mask; }

// (i, j), i < j, of pair index t in [0, n(n-1)/2): i from the root of
// i^2 - (2n - 1) i + 2t = 0 in FP64, then moved by whole rows until
// start(i) <= t < start(i + 1), start(i) = i n - i(i+1)/2 (exact integers).
__device__ __forceinline__ void er_unrank(uint64_t t, int64_t n, int64_t* pi, int64_t* pj) {
  const double b = 2.0 * (double)n - 1.0;
  int64_t i = (int64_t)((b - sqrt(fmax(b * b - 8.0 * (double)t, 0.0))) * 0.5);
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  auto start = [n](int64_t r) { return (uint64_t)(r * n - r * (r + 1) / 2); };
  while (i > 0 && start(i) > t) --i;
  while (i < n - 2 && start(i + 1) <= t) ++i;
  *pi = i;
  *pj = (int64_t)(t - start(i)) + i + 1;
}

__global__ __launch_bounds__(kGenNT) void k_er_clear(uint64_t P, uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ idx) {
  const uint64_t stride = (uint64_t)gridDim.x * kGenNT;
  for (uint64_t q = (uint64_t)blockIdx.x * kGenNT + threadIdx.x; q < P; q += stride) {
    keys[q] = kErEmpty;
    idx[q] = kErNoIdx;
  }
}

__global__ __launch_bounds__(kGenNT) void k_er_insert(int64_t K, uint64_t N, uint64_t S, uint64_t mask,
                                                      uint64_t* __restrict__ keys, uint32_t* __restrict__ idx) {
  const int64_t stride = (int64_t)gridDim.x * kGenNT;
  for (int64_t k = (int64_t)blockIdx.x * kGenNT + threadIdx.x; k < K; k += stride) {
    const uint64_t x = __umul64hi(er_word(S, (uint64_t)k), N);
    uint64_t q = er_slot(x, mask);
    while (true) {  // the table is at most half full, so a free slot or x is always reached
      const unsigned long long prev = atomicCAS(reinterpret_cast<unsigned long long*>(&keys[q]), kErEmpty, x);
      if (prev == kErEmpty || prev == x) {
        atomicMin(&idx[q], (uint32_t)k);
        break;
      }
      q = (q + 1) & mask;
    }
  }
}

// flag[k] = 1 when draw k is the first draw of its value.
__global__ __launch_bounds__(kGenNT) void k_er_flag(int64_t K, uint64_t N, uint64_t S, uint64_t mask,
                                                    const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ idx, int32_t* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * kGenNT;
  for (int64_t k = (int64_t)blockIdx.x * kGenNT + threadIdx.x; k < K; k += stride) {
    const uint64_t x = __umul64hi(er_word(S, (uint64_t)k), N);
    uint64_t q = er_slot(x, mask);
    while (keys[q] != x) q = (q + 1) & mask;
    flag[k] = idx[q] == (uint32_t)k;
  }
}

// New draw k with pos[k] < m becomes edge pos[k].
__global__ __launch_bounds__(kGenNT) void k_er_emit(int64_t K, int64_t n, uint64_t N, uint64_t S, int64_t m,
                                                    const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                                                    int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * kGenNT;
  for (int64_t k = (int64_t)blockIdx.x * kGenNT + threadIdx.x; k < K; k += stride) {
    const int64_t e = pos[k];
    if (!flag[k] || e >= m) continue;
    const uint64_t w = er_word(S, (uint64_t)k);
    int64_t i, j;
    er_unrank(__umul64hi(w, N), n, &i, &j);
    if (w & 1u) {
      src[e] = (int32_t)j;
      dst[e] = (int32_t)i;
    } else {
      src[e] = (int32_t)i;
      dst[e] = (int32_t)j;
    }
  }
}

// ---------------------------------------------------------------------------
// Barabasi-Albert (the paper's generator table, Section 4): nodes 0..k form
// the seed clique K_{k+1} (its edges in lexicographic (i, j) order); node v > k
// then adds edges e = E_v + j, j = 0..k-1, E_v = k(k+1)/2 + (v - k - 1) k,
// each from v to a node drawn with probability proportional to its degree
// among the edges before E_v: a position r uniform in [0, 2 E_v) of the
// endpoint list (edge e' holds its source at 2e' and its target at 2e' + 1),
// r = floor(word((e << 20) + a + 1) 2 E_v / 2^64) with S = out(seed + 14
// gamma), attempt a = 0, 1, ...; a draw equal to a target v already took
// is redrawn with the next attempt, so v's k targets are distinct. Targets
// at odd positions are other edges' targets: each pass resolves every edge
// whose draws only reach edges already final (they never change), until
// none is left; the earliest unresolved edge only reaches final edges, so
// every pass makes progress.

__device__ __forceinline__ void ba_seed_pair(int64_t e, int32_t k, int32_t* pi, int32_t* pj) {
  int32_t i = 0;
  int64_t row = k;  // pairs (i, i+1 .. k)
  while (e >= row) {
    e -= row;
    ++i;
    --row;
  }
  *pi = i;
  *pj = i + 1 + (int32_t)e;
}

__global__ __launch_bounds__(kGenNT) void k_ba_init(int64_t m, int32_t k, int64_t e_seed, int32_t* __restrict__ src,
                                                    int32_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * kGenNT;
  for (int64_t e = (int64_t)blockIdx.x * kGenNT + threadIdx.x; e < m; e += stride) {
    if (e < e_seed) {
      int32_t i, j;
      ba_seed_pair(e, k, &i, &j);
      src[e] = i;
      dst[e] = j;
    } else {
      src[e] = (int32_t)(k + 1 + (e - e_seed) / k);
      dst[e] = -1;
    }
  }
}

constexpr int32_t kBaMaxAttempts = 1 << 20;

// One pass over the nodes v > k still unresolved (prog[v] = next slot j in
// the low 8 bits, attempt a above; k <= 255). pending counts the nodes left; err is
// set if some edge runs out of attempts.
__global__ __launch_bounds__(kGenNT) void k_ba_pass(int32_t n, int32_t k, int64_t e_seed, uint64_t S,
                                                    const int32_t* __restrict__ src, int32_t* __restrict__ dst,
                                                    int32_t* __restrict__ prog, int32_t* __restrict__ pending,
                                                    int32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * kGenNT;
  int32_t left = 0;
  for (int64_t v = (int64_t)k + 1 + (int64_t)blockIdx.x * kGenNT + threadIdx.x; v < n; v += stride) {
    int32_t p = prog[v];
    int32_t j = p & 0xFF, a = p >> 8;
    if (j >= k) continue;
    const int64_t ev = e_seed + (v - k - 1) * (int64_t)k;
    const uint64_t span = 2u * (uint64_t)ev;
    while (j < k) {
      const int64_t e = ev + j;
      const uint64_t r = __umul64hi(sm64(S + kGamma * (((uint64_t)e << 20) + (uint64_t)a + 1u)), span);
      const int64_t e2 = (int64_t)(r >> 1);
      int32_t c;
      if ((r & 1u) == 0) {
        c = src[e2];
      } else {
        c = __atomic_load_n(&dst[e2], __ATOMIC_RELAXED);
        if (c < 0) break;  // that edge is not final yet: next pass
      }
      bool dup = false;
      for (int32_t q = 0; q < j; ++q) dup |= dst[ev + q] == c;
      if (dup) {
        if (++a >= kBaMaxAttempts) {
          atomicOr(err, 1);
          j = k;
          break;
        }
        continue;
      }
      __atomic_store_n(&dst[e], c, __ATOMIC_RELAXED);
      ++j;
      a = 0;
    }
    prog[v] = j | (a << 8);
    left += j < k;
  }
  #pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) left += __shfl_xor(left, o, kWave);
  if (lane_id() == 0 && left) atomicAdd(pending, left);
}

__global__ __launch_bounds__(kGenNT) void k_ba_zero(int32_t n, int32_t* __restrict__ prog, int32_t* __restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * kGenNT;
  for (int64_t v = (int64_t)blockIdx.x * kGenNT + threadIdx.x; v < n; v += stride) prog[v] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 2) cnt[threadIdx.x] = 0;
}

__global__ void k_ba_reset(int32_t* __restrict__ pending) {
  if (threadIdx.x == 0) *pending = 0;
}

unsigned gen_grid(int64_t work) {
  const int64_t b = (work + kGenNT - 1) / kGenNT;
  return (unsigned)(b < 1 ? 1 : b > 65536 ? 65536 : b);
}

}  // namespace

hipError_t launch_gen_rmat(int64_t m, int scale, const double abcd[4], double noise, uint64_t seed,
                           const int32_t* perm, int32_t* src, int32_t* dst, hipStream_t s) {
  if (m > 0) {
    const int64_t blocks = (m + kGenNT - 1) / kGenNT;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    k_gen_rmat<<<grid, kGenNT, 0, s>>>(m, scale, abcd[0], abcd[1], abcd[2], abcd[3], noise, seed, perm, src, dst);
  }
  return hipGetLastError();
}

}  // namespace tricc

namespace tricc {

hipError_t launch_er_clear(uint64_t P, uint64_t* keys, uint32_t* idx, hipStream_t s) {
  k_er_clear<<<gen_grid((int64_t)P), kGenNT, 0, s>>>(P, keys, idx);
  return hipGetLastError();
}

hipError_t launch_er_insert(int64_t K, uint64_t N, uint64_t seed, uint64_t mask, uint64_t* keys, uint32_t* idx,
                            hipStream_t s) {
  if (K <= 0) return hipSuccess;
  k_er_insert<<<gen_grid(K), kGenNT, 0, s>>>(K, N, sm64_host(seed + kGamma * 13u), mask, keys, idx);
  return hipGetLastError();
}

hipError_t launch_er_flag(int64_t K, uint64_t N, uint64_t seed, uint64_t mask, const uint64_t* keys,
                          const uint32_t* idx, int32_t* flag, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  k_er_flag<<<gen_grid(K), kGenNT, 0, s>>>(K, N, sm64_host(seed + kGamma * 13u), mask, keys, idx, flag);
  return hipGetLastError();
}

hipError_t launch_er_emit(int64_t K, int64_t n, uint64_t N, uint64_t seed, int64_t m, const int32_t* flag,
                          const int64_t* pos, int32_t* src, int32_t* dst, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  k_er_emit<<<gen_grid(K), kGenNT, 0, s>>>(K, n, N, sm64_host(seed + kGamma * 13u), m, flag, pos, src, dst);
  return hipGetLastError();
}

hipError_t launch_ba_init(int64_t m, int32_t k, int32_t n, int32_t* src, int32_t* dst, int32_t* prog, int32_t* cnt,
                          hipStream_t s) {
  const int64_t e_seed = (int64_t)k * (k + 1) / 2;
  if (m > 0) k_ba_init<<<gen_grid(m), kGenNT, 0, s>>>(m, k, e_seed, src, dst);
  k_ba_zero<<<gen_grid(n), kGenNT, 0, s>>>(n, prog, cnt);
  return hipGetLastError();
}

hipError_t launch_ba_pass(int32_t n, int32_t k, uint64_t seed, const int32_t* src, int32_t* dst, int32_t* prog,
                          int32_t* cnt, hipStream_t s) {
  const int64_t e_seed = (int64_t)k * (k + 1) / 2;
  k_ba_reset<<<1, 64, 0, s>>>(cnt);
  const int64_t work = (int64_t)n - k - 1;
  if (work > 0)
    k_ba_pass<<<gen_grid(work), kGenNT, 0, s>>>(n, k, e_seed, sm64_host(seed + kGamma * 14u), src, dst, prog, cnt,
                                               cnt + 1);
  return hipGetLastError();
}

}  // namespace tricc

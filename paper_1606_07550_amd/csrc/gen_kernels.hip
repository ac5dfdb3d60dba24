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

__device__ __forceinline__ uint64_t sm64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

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

// 4-clique counts (clique detection, among the graph-motif methods of
// Section 4): the triangle method one size up on the same degree-ordered
// DAG. A 4-clique u < w < x < z (by rank) is met once, at u: w in N+(u),
// x in C = N+(u) ∩ N+(w), z in N+(x) ∩ C.
#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

constexpr int kK4NT = 256;
constexpr int kK4Waves = kK4NT / kWave;

// First position p in L[0, d) (ascending) with L[p] >= x.
__device__ __forceinline__ int32_t lower_pos(const int32_t* L, int32_t d, int32_t x) {
  int32_t lo = 0, hi = d;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (L[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One block per node u (grid-stride over the ids); each wavefront takes the
// out-neighbours w of u in turn: it lists C_w = N+(w) ∩ N+(u) in id order
// (each id of N+(w) searched in N+(u), held sorted in LDS), then streams the
// out-lists of the x in C_w packed (a window of up to 64 lists in the lanes,
// each step one id per lane) and counts the ids z found in C_w. Exactly
// 40 KB of LDS per block, so four blocks share a CU.
template <int CAP>
__global__ __launch_bounds__(kK4NT) void k_count_k4(int32_t n, const int64_t* __restrict__ doff,
                                                    const int32_t* __restrict__ dcol,
                                                    unsigned long long* __restrict__ total) {
  __shared__ __align__(16) int32_t L[CAP];
  __shared__ int32_t Cl[kK4Waves][CAP];
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  unsigned long long acc = 0;
  for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {  // block-uniform
    const int64_t ub = doff[u];
    const int32_t d = (int32_t)(doff[u + 1] - ub);
    if (d < 3) continue;
    __syncthreads();  // L of the previous node is no longer read
    for (int32_t i = threadIdx.x; i < d; i += kK4NT) L[i] = dcol[ub + i];
    __syncthreads();
    for (int32_t i = wv; i < d; i += kK4Waves) {  // w = L[i]
      const int32_t w = L[i];
      const int64_t wb = doff[w];
      const int32_t dw = (int32_t)(doff[w + 1] - wb);
      int32_t nc = 0;  // wave-uniform
      for (int32_t t0 = 0; t0 < dw; t0 += kWave) {
        const int32_t t = t0 + lane;
        bool hit = false;
        int32_t y = 0;
        if (t < dw) {
          y = dcol[wb + t];
          const int32_t p = lower_pos(L, d, y);
          hit = p < d && L[p] == y;
        }
        const uint64_t m = __ballot(hit);
        if (hit) Cl[wv][nc + mask_below(m)] = y;
        nc += (int32_t)__popcll(m);
      }
      wave_sync();
      const int32_t* C = Cl[wv];
      // edges x -> z inside C_w, over the out-lists of the x in C_w (a
      // clique needs two of them)
      for (int32_t base = 0; nc >= 2 && base < nc; base += kWave) {
        int32_t xn = 0, xb = 0;
        if (base + lane < nc) {
          const int32_t x = C[base + lane];
          const int64_t b = doff[x];
          xb = (int32_t)b;
          xn = (int32_t)(doff[x + 1] - b);
        }
        const int32_t incl = wave_incl_scan(xn);
        const int32_t tot = __shfl(incl, kWave - 1, kWave);
        const int32_t excl = incl - xn;
        for (int32_t t0 = 0; t0 < tot; t0 += kWave) {
          const int32_t t = t0 + lane;
          int k = 0;
#pragma unroll
          for (int s = kWave / 2; s > 0; s >>= 1) {
            const int32_t v = __shfl(incl, k + s - 1, kWave);
            if (v <= t) k += s;
          }
          const int32_t kb = __shfl(xb, k, kWave);
          const int32_t ke = __shfl(excl, k, kWave);
          if (t < tot) {
            const int32_t z = dcol[kb + (t - ke)];
            const int32_t p = lower_pos(C, nc, z);
            if (p < nc && C[p] == z) ++acc;
          }
        }
      }
      wave_sync();  // the next w reuses Cl
    }
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  unsigned long long* red = reinterpret_cast<unsigned long long*>(L);  // L is free now
  __syncthreads();
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < kK4Waves; ++q) t += red[q];
    if (t) atomicAdd(total, t);
  }
}

__global__ void k_zero_one(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0ull;
}

}  // namespace

hipError_t launch_count_k4(int32_t n, const int64_t* doff, const int32_t* dcol, unsigned long long* total,
                           hipStream_t s) {
  k_zero_one<<<1, 64, 0, s>>>(total);
  if (n > 0) {
    const unsigned grid = (unsigned)(n < 65536 ? n : 65536);
    k_count_k4<kK4Cap><<<grid, kK4NT, 0, s>>>(n, doff, dcol, total);
  }
  return hipGetLastError();
}

}  // namespace tricc

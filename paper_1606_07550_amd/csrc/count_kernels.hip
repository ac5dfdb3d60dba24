// Intersection kernels (the hot loop) and the clustering-coefficient
// epilogue for gfx950.
//
// Every triangle {u, w, x} with rank(u) < rank(w) < rank(x) (rank = (d, id))
// is met exactly once: at the DAG edge u->w, as a common element x of the
// out-lists N+(u) and N+(w). The work unit is a node u: its out-list is
// staged in LDS as an open-addressing hash table whose slots also carry a
// counter, the out-lists N+(w) of its out-neighbours are streamed from HBM
// (consecutive lanes read consecutive ids) and probed against the table.
// A hit on x credits x and w in the LDS counters; u gets the number of hits.
// The counters are flushed with one 64-bit atomic per out-neighbour at the
// end, so no atomic is issued per triangle. The edge test of the paper's
// complexity table (binary search in a sorted vector, Section 5.1) becomes a
// hash probe in LDS; the fallback kernel for out-lists too large for LDS
// keeps the binary search, in global memory.
//
// Nodes are binned by d+(u); a bin's variant fixes the lane-group size G
// that owns one node, the sub-group size SG that streams one N+(w), and the
// table size SLOTS (at most half full).
#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

template <int G>
__device__ __forceinline__ void group_sync() {
  if constexpr (G > kWave) __syncthreads();
  else wave_sync();
}

template <int SLOTS>
__device__ __forceinline__ int table_find(const int32_t* K, int32_t x) {
  constexpr int bits = __builtin_ctz(SLOTS);
  uint32_t h = hash_slot(x, bits);
  while (true) {
    const int32_t k = K[h];
    if (k == x) return (int)h;
    if (k < 0) return -1;
    h = (h + 1) & (SLOTS - 1);
  }
}

template <int SLOTS>
__device__ __forceinline__ void table_insert(int32_t* K, int32_t x) {
  constexpr int bits = __builtin_ctz(SLOTS);
  uint32_t h = hash_slot(x, bits);
  while (atomicCAS(&K[h], -1, x) != -1) h = (h + 1) & (SLOTS - 1);
}

}  // namespace

// NT threads per block; groups of G lanes (G divides NT, or G == NT).
template <int NT, int G, int SG, int SLOTS>
__global__ __launch_bounds__(NT) void k_count_hash(const int32_t* __restrict__ list, int32_t nlist,
                                                   const int64_t* __restrict__ doff,
                                                   const int32_t* __restrict__ dcol,
                                                   unsigned long long* __restrict__ T) {
  static_assert(NT % G == 0 && G % SG == 0 && SG <= kWave, "shape");
  constexpr int GPB = NT / G;
  constexpr int NSUB = G / SG;
  __shared__ int32_t Ks[GPB][SLOTS];
  __shared__ uint32_t Cs[GPB][SLOTS];
  __shared__ unsigned long long red[NT / kWave];
  const int gi = threadIdx.x / G;
  const int g = threadIdx.x % G;
  const int idx = blockIdx.x * GPB + gi;
  int32_t* K = Ks[gi];
  uint32_t* C = Cs[gi];
  const bool active = idx < nlist;
  unsigned long long tu = 0;
  int32_t u = 0;
  if (active) {
    u = list[idx];
    const int64_t beg = doff[u];
    const int32_t len = (int32_t)(doff[u + 1] - beg);
    for (int s = g; s < SLOTS; s += G) { K[s] = -1; C[s] = 0; }
    group_sync<G>();
    for (int i = g; i < len; i += G) table_insert<SLOTS>(K, dcol[beg + i]);
    group_sync<G>();
    const int sub = g / SG, sg = g % SG;
    for (int i = sub; i < len; i += NSUB) {
      const int32_t w = dcol[beg + i];
      const int64_t wb = doff[w], we = doff[w + 1];
      uint32_t cw = 0;
      for (int64_t p = wb + sg; p < we; p += SG) {
        const int s = table_find<SLOTS>(K, dcol[p]);
        if (s >= 0) { atomicAdd(&C[s], 1u); ++cw; }
      }
      if (cw) atomicAdd(&C[table_find<SLOTS>(K, w)], cw);
      tu += cw;
    }
    group_sync<G>();
    for (int s = g; s < SLOTS; s += G) {
      const int32_t k = K[s];
      const uint32_t c = C[s];
      if (k >= 0 && c) atomicAdd(&T[k], (unsigned long long)c);
    }
  }
  if constexpr (G <= kWave) {
    tu = group_sum<unsigned long long, G>(tu);
    if (active && g == 0 && tu) atomicAdd(&T[u], tu);
  } else {
    const unsigned long long t = block_sum<unsigned long long, NT>(tu, red);
    if (threadIdx.x == 0 && active && t) atomicAdd(&T[u], t);
  }
}

// Fallback for out-lists of any length: one block per node, N+(u) stays in
// global memory and is binary-searched; hits are credited with global atomics.
__global__ __launch_bounds__(256) void k_count_global(const int32_t* __restrict__ list, int32_t nlist,
                                                      const int64_t* __restrict__ doff,
                                                      const int32_t* __restrict__ dcol,
                                                      unsigned long long* __restrict__ T) {
  __shared__ unsigned long long red[256 / kWave];
  const int32_t u = list[blockIdx.x];
  const int64_t beg = doff[u];
  const int32_t len = (int32_t)(doff[u + 1] - beg);
  const int32_t* U = dcol + beg;
  const int wv = threadIdx.x / kWave, l = lane_id();
  unsigned long long tu = 0;
  for (int i = wv; i < len; i += 256 / kWave) {
    const int32_t w = U[i];
    const int64_t wb = doff[w], we = doff[w + 1];
    unsigned long long cw = 0;
    for (int64_t p = wb + l; p < we; p += kWave) {
      const int32_t x = dcol[p];
      int32_t lo = 0, hi = len;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (U[mid] < x) lo = mid + 1; else hi = mid;
      }
      if (lo < len && U[lo] == x) { atomicAdd(&T[x], 1ull); ++cw; }
    }
    cw = group_sum<unsigned long long, kWave>(cw);  // every lane now holds the wave total
    if (l == 0) {
      if (cw) atomicAdd(&T[w], cw);
      tu += cw;
    }
  }
  const unsigned long long t = block_sum<unsigned long long, 256>(tu, red);
  if (threadIdx.x == 0 && t) atomicAdd(&T[u], t);
}

// ---------------------------------------------------------------------------
// Variant table. Capacity = SLOTS / 2 (table at most half full).
struct VariantInfo { int nt, g, sg, slots; };
static constexpr VariantInfo kVariants[] = {
    {256, 16, 16, 32},      // 0: d+ <= 16
    {256, 16, 8, 32},       // 1
    {256, 64, 64, 128},     // 2: d+ <= 64
    {256, 64, 32, 128},     // 3
    {256, 64, 16, 128},     // 4
    {256, 64, 64, 512},     // 5: d+ <= 256
    {256, 64, 32, 512},     // 6
    {256, 64, 16, 512},     // 7
    {256, 256, 64, 2048},   // 8: d+ <= 1024
    {256, 256, 32, 2048},   // 9
    {256, 256, 16, 2048},   // 10
    {512, 512, 64, 8192},   // 11: d+ <= 4096
    {512, 512, 32, 8192},   // 12
    {1024, 1024, 64, 16384},  // 13: d+ <= 8192 (128 KiB LDS)
    {256, 256, 64, 0},      // 14: global fallback, any d+
};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kVariantGlobal = kNumVariants - 1;

int count_variant_valid(int v) { return v >= 0 && v < kNumVariants; }
int count_variant_capacity(int v) {
  if (!count_variant_valid(v)) return -1;
  return kVariants[v].slots ? kVariants[v].slots / 2 : 0x7fffffff;
}

template <int NT, int G, int SG, int SLOTS>
static void launch_hash(const BinLaunch& b, const int64_t* doff, const int32_t* dcol,
                        unsigned long long* T, hipStream_t s) {
  constexpr int GPB = NT / G;
  const unsigned grid = (unsigned)((b.count + GPB - 1) / GPB);
  k_count_hash<NT, G, SG, SLOTS><<<grid, NT, 0, s>>>(b.list, b.count, doff, dcol, T);
}

hipError_t launch_count_bin(const BinLaunch& b, const int64_t* doff, const int32_t* dcol,
                            unsigned long long* T, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  switch (b.variant) {
    case 0: launch_hash<256, 16, 16, 32>(b, doff, dcol, T, s); break;
    case 1: launch_hash<256, 16, 8, 32>(b, doff, dcol, T, s); break;
    case 2: launch_hash<256, 64, 64, 128>(b, doff, dcol, T, s); break;
    case 3: launch_hash<256, 64, 32, 128>(b, doff, dcol, T, s); break;
    case 4: launch_hash<256, 64, 16, 128>(b, doff, dcol, T, s); break;
    case 5: launch_hash<256, 64, 64, 512>(b, doff, dcol, T, s); break;
    case 6: launch_hash<256, 64, 32, 512>(b, doff, dcol, T, s); break;
    case 7: launch_hash<256, 64, 16, 512>(b, doff, dcol, T, s); break;
    case 8: launch_hash<256, 256, 64, 2048>(b, doff, dcol, T, s); break;
    case 9: launch_hash<256, 256, 32, 2048>(b, doff, dcol, T, s); break;
    case 10: launch_hash<256, 256, 16, 2048>(b, doff, dcol, T, s); break;
    case 11: launch_hash<512, 512, 64, 8192>(b, doff, dcol, T, s); break;
    case 12: launch_hash<512, 512, 32, 8192>(b, doff, dcol, T, s); break;
    case 13: launch_hash<1024, 1024, 64, 16384>(b, doff, dcol, T, s); break;
    case kVariantGlobal:
      k_count_global<<<(unsigned)b.count, 256, 0, s>>>(b.list, b.count, doff, dcol, T);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  k_zero_u64<<<(unsigned)g, 256, 0, s>>>(p, n);
  return hipGetLastError();
}

// a7: CC(v) = 2T(v) / (d(v)(d(v)-1)) for d >= 2, else 0. The ratio is formed
// in FP64 from exact integers (both below 2^53) and rounded once to FP32.
// Each block owns a fixed range of nodes and reduces it in a fixed order, so
// the FP64 sum (and the average) does not depend on scheduling.
constexpr int kEpiThreads = 256;
constexpr int kEpiItems = 16;
int64_t epilogue_blocks(int64_t n) { return (n + kEpiThreads * kEpiItems - 1) / (kEpiThreads * kEpiItems); }

__global__ __launch_bounds__(kEpiThreads) void k_epilogue(int32_t n, const unsigned long long* __restrict__ T,
                                                          const int32_t* __restrict__ deg,
                                                          float* __restrict__ cc, double* __restrict__ part_cc,
                                                          unsigned long long* __restrict__ part_T) {
  __shared__ double red_d[kEpiThreads / kWave];
  __shared__ unsigned long long red_t[kEpiThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kEpiThreads * kEpiItems;
  double acc = 0.0;
  unsigned long long tacc = 0;
#pragma unroll 4
  for (int k = 0; k < kEpiItems; ++k) {
    const int64_t v = base + (int64_t)k * kEpiThreads + threadIdx.x;
    if (v >= n) break;
    const unsigned long long t = T[v];
    const int64_t d = deg[v];
    double r = 0.0;
    if (d >= 2) r = (2.0 * (double)t) / ((double)d * (double)(d - 1));
    cc[v] = (float)r;
    acc += r;
    tacc += t;
  }
  const double s = block_sum<double, kEpiThreads>(acc, red_d);
  const unsigned long long st = block_sum<unsigned long long, kEpiThreads>(tacc, red_t);
  if (threadIdx.x == 0) { part_cc[blockIdx.x] = s; part_T[blockIdx.x] = st; }
}

__global__ __launch_bounds__(256) void k_finish(int64_t nb, int32_t n, const double* __restrict__ part_cc,
                                                const unsigned long long* __restrict__ part_T,
                                                unsigned long long* __restrict__ total, double* __restrict__ avg) {
  __shared__ double red_d[256 / kWave];
  __shared__ unsigned long long red_t[256 / kWave];
  double acc = 0.0;
  unsigned long long tacc = 0;
  for (int64_t i = threadIdx.x; i < nb; i += 256) { acc += part_cc[i]; tacc += part_T[i]; }
  const double s = block_sum<double, 256>(acc, red_d);
  const unsigned long long st = block_sum<unsigned long long, 256>(tacc, red_t);
  if (threadIdx.x == 0) {
    *total = st / 3ull;
    *avg = n > 0 ? s / (double)n : 0.0;
  }
}

hipError_t launch_epilogue(int32_t n, const unsigned long long* T, const int32_t* deg, float* cc,
                           double* part_cc, unsigned long long* part_T, hipStream_t s) {
  const int64_t nb = epilogue_blocks(n);
  if (nb == 0) return hipSuccess;
  k_epilogue<<<(unsigned)nb, kEpiThreads, 0, s>>>(n, T, deg, cc, part_cc, part_T);
  return hipGetLastError();
}

hipError_t launch_finish(int64_t nb, int32_t n, const double* part_cc, const unsigned long long* part_T,
                         unsigned long long* total, double* avg, hipStream_t s) {
  k_finish<<<1, 256, 0, s>>>(nb, n, part_cc, part_T, total, avg);
  return hipGetLastError();
}

}  // namespace tricc

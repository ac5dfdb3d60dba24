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
// Out-degrees up to kK4BitsMid take the bit-row kernel with 256 threads and
// 38 KB of LDS; up to kK4BitsMax the one with 1,024 threads and 132 KB (one
// block per CU); longer lists the list kernel.
constexpr int kK4BitsMid = 512;
constexpr int kK4BitsMax = 1024;

// Position of the first element >= x in L[0, P), P a power of two and L
// ascending (padded past its length with kPad, above every id): fixed
// halving steps, no data-dependent exit. Every element before the result is
// below x, so x is in L iff L[result] == x.
__device__ __forceinline__ int32_t pow2_lower_pos(const int32_t* L, int32_t P, int32_t x) {
  int32_t p = 0;
  for (int32_t s = P >> 1; s > 0; s >>= 1)
    if (L[p + s - 1] < x) p += s;
  return p;
}

// One (u, w) pair, one wavefront: lists C_w = N+(w) ∩ N+(u) into C in id
// order (each id of N+(w) searched in N+(u), held sorted in L and padded with
// kPad to the power of two P), then streams the out-lists of the x in C_w
// packed (a window of up to 64 lists in the lanes, each step one id per lane)
// and counts the ids z found in C_w: the 4-cliques {u, w, x, z}. C holds up
// to P ids. Returns this lane's share.
__device__ __forceinline__ unsigned long long wave_k4_pair(const int32_t* L, int32_t P, int32_t w, int32_t* C,
                                                           const int64_t* __restrict__ doff,
                                                           const int32_t* __restrict__ dcol, int lane) {
  const int64_t wb = doff[w];
  const int32_t dw = (int32_t)(doff[w + 1] - wb);
  if (dw < 2) return 0;  // a clique needs two ids of N+(w) in C_w
  unsigned long long acc = 0;
  int32_t nc = 0;  // wave-uniform
  for (int32_t t0 = 0; t0 < dw; t0 += kWave) {
    const int32_t t = t0 + lane;
    bool hit = false;
    int32_t y = 0;
    if (t < dw) {
      y = dcol[wb + t];
      hit = L[pow2_lower_pos(L, P, y)] == y;
    }
    const uint64_t m = __ballot(hit);
    if (hit) C[nc + mask_below(m)] = y;
    nc += (int32_t)__popcll(m);
  }
  // pad C_w to a power of two for the fixed-step search (nc <= d <= the capacity of C)
  const int32_t Pc = nc <= 1 ? 1 : 1 << (32 - __builtin_clz((uint32_t)(nc - 1)));
  for (int32_t t = nc + lane; t < Pc; t += kWave) C[t] = kPad;
  wave_sync();
  for (int32_t base = 0; nc >= 2 && base < nc; base += kWave) {
    int32_t xn = 0;
    int64_t xb = 0;  // start of N+(x): DAG offsets pass 2^31 on large graphs
    if (base + lane < nc) {
      const int32_t x = C[base + lane];
      const int64_t b = doff[x];
      xb = b;
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
      const int64_t kb = __shfl(xb, k, kWave);
      const int32_t ke = __shfl(excl, k, kWave);
      if (t < tot) {
        const int32_t z = dcol[kb + (t - ke)];
        if (C[pow2_lower_pos(C, Pc, z)] == z) ++acc;
      }
    }
  }
  wave_sync();  // the next pair reuses C
  return acc;
}

// Block-wide total of the per-lane counts, one 64-bit atomic per block.
// `red` holds NW values (the block's wavefronts); contains __syncthreads().
template <int NW>
__device__ __forceinline__ void k4_block_total(unsigned long long acc, unsigned long long* red,
                                               unsigned long long* total) {
  const int wv = threadIdx.x / kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  __syncthreads();
  if (lane_id() == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < NW; ++q) t += red[q];
    if (t) atomicAdd(total, t);
  }
}

// Nodes with DMIN < d+(u) <= DMAX (and d+(u) >= 3): one block of NT threads
// per node. The block scans `chunk` (<= NT) consecutive ids at a time
// (grid-stride over such chunks), queues the ones in range in LDS, then
// takes them in turn. The block builds the subgraph induced on N+(u) as bit rows in
// LDS (row i: the positions in N+(u) of N+(L[i]) ∩ N+(u), each wavefront
// building the rows of its w's by searching N+(w) in N+(u)); then every pair
// (w, x) with x in row w adds popcount(row w & row x): the z that close the
// 4-clique {u, w, x, z}. Rows take RS = 2^rs words (RS >= d / 32), and the
// lanes of a wavefront cover 64 / RS rows x at once, one word each. LISTED:
// the x of row w are first listed in LDS by ballot; otherwise (rows of 32
// words, DMIN >= 512) they are taken two at a time straight from row w's
// bits, which leaves the LDS for 1,024 threads.
template <int DMIN, int DMAX, int NT, bool LISTED>
__global__ __launch_bounds__(NT) void k_count_k4_bits(int32_t n, int32_t chunk, const int64_t* __restrict__ doff,
                                                      const int32_t* __restrict__ dcol,
                                                      unsigned long long* __restrict__ total) {
  constexpr int NW = NT / kWave;
  static_assert(DMAX % 32 == 0 && DMAX <= 65536, "positions are stored in 16 bits");
  static_assert(LISTED || (DMIN >= 512 && DMAX <= 1024), "unlisted rows must be 32 words");
  __shared__ int32_t L[DMAX];
  __shared__ uint32_t B[DMAX * (DMAX / 32)];
  __shared__ uint16_t Pl[LISTED ? NW : 1][LISTED ? DMAX : 1];
  __shared__ unsigned long long red[NW];
  __shared__ int32_t Q[NT];
  __shared__ int32_t Qn;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  unsigned long long acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * chunk; base < n; base += (int64_t)gridDim.x * chunk) {
    __syncthreads();  // the previous chunk's queue has been taken
    if (threadIdx.x == 0) Qn = 0;
    __syncthreads();
    const int64_t v = base + threadIdx.x;
    if ((int)threadIdx.x < chunk && v < n) {
      const int32_t dv = (int32_t)(doff[v + 1] - doff[v]);
      if (dv >= 3 && dv > DMIN && dv <= DMAX) Q[atomicAdd(&Qn, 1)] = (int32_t)v;
    }
    __syncthreads();
    const int32_t nq = Qn;
    for (int32_t qi = 0; qi < nq; ++qi) {  // block-uniform
      const int32_t u = Q[qi];
      const int64_t ub = doff[u];
      const int32_t d = (int32_t)(doff[u + 1] - ub);
      const int rs = d <= 32 ? 0 : 32 - __builtin_clz((uint32_t)((d + 31) / 32 - 1));
      const int RS = 1 << rs;
      const int32_t P = 1 << (32 - __builtin_clz((uint32_t)(d - 1)));  // power of two >= d, <= DMAX
      __syncthreads();  // L and B of the previous node are no longer read
      for (int32_t i = threadIdx.x; i < P; i += NT) L[i] = i < d ? dcol[ub + i] : kPad;
      for (int32_t q = threadIdx.x; q < d * RS; q += NT) B[q] = 0u;
      __syncthreads();
      for (int32_t i = wv; i < d; i += NW) {
        const int32_t w = L[i];
        const int64_t wb = doff[w];
        const int32_t dw = (int32_t)(doff[w + 1] - wb);
        for (int32_t t = lane; t < dw; t += kWave) {
          const int32_t y = dcol[wb + t];
          const int32_t p = pow2_lower_pos(L, P, y);
          if (L[p] == y) atomicOr(&B[i * RS + (p >> 5)], 1u << (p & 31));
        }
      }
      __syncthreads();
      for (int32_t i = wv; i < d && !LISTED; i += NW) {
        // RS == 32: half-wave h takes the h-th of each next two bits of row i
        const uint32_t* Bi = B + i * 32;
        const int32_t k = lane & 31;
        const bool second = lane >= 32;
        const uint32_t bik = Bi[k];
        int32_t kw = 0;
        uint32_t word = Bi[0];
        while (true) {
          while (word == 0u && kw < 31) word = Bi[++kw];
          if (word == 0u) break;
          const int32_t xa = kw * 32 + __builtin_ctz(word);
          word &= word - 1u;
          while (word == 0u && kw < 31) word = Bi[++kw];
          const int32_t xb = word ? kw * 32 + __builtin_ctz(word) : -1;
          word &= word - 1u;  // no effect when word == 0
          const int32_t x = second ? xb : xa;
          if (x >= 0) acc += (unsigned long long)__popc(bik & B[x * 32 + k]);
          if (xb < 0) break;
        }
      }
      for (int32_t i = wv; i < d && LISTED; i += NW) {
        const uint32_t* Bi = B + i * RS;
        int32_t np = 0;  // wave-uniform: the x of row i, listed
        for (int32_t b0 = 0; b0 < d; b0 += kWave) {
          const int32_t b = b0 + lane;
          const bool bit = b < d && ((Bi[b >> 5] >> (b & 31)) & 1u);
          const uint64_t m = __ballot(bit);
          if (bit) Pl[wv][np + mask_below(m)] = (uint16_t)b;
          np += (int32_t)__popcll(m);
        }
        wave_sync();
        if (np >= 2) {  // a clique needs x and z in row i
          const int32_t k = lane & (RS - 1);
          const int32_t js = lane >> rs;
          const uint32_t bik = Bi[k];
          for (int32_t j0 = 0; j0 < np; j0 += (kWave >> rs)) {
            const int32_t jj = j0 + js;
            if (jj < np) acc += (unsigned long long)__popc(bik & B[(int32_t)Pl[wv][jj] * RS + k]);
          }
        }
        wave_sync();  // the next row reuses Pl
      }
    }
  }
  k4_block_total<NW>(acc, red, total);
}

// Nodes with d+(u) > kK4BitsMax: one block per node (chunks of ids scanned
// and queued as in the bit-row kernel), N+(u) in LDS, the wavefronts taking
// its out-neighbours w in turn.
template <int CAP>
__global__ __launch_bounds__(kK4NT) void k_count_k4(int32_t n, int32_t chunk, const int64_t* __restrict__ doff,
                                                    const int32_t* __restrict__ dcol,
                                                    unsigned long long* __restrict__ total) {
  __shared__ __align__(16) int32_t L[CAP];
  __shared__ int32_t Cl[kK4Waves][CAP];
  __shared__ int32_t Q[kK4NT];
  __shared__ int32_t Qn;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  unsigned long long acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * chunk; base < n; base += (int64_t)gridDim.x * chunk) {
    __syncthreads();  // the previous chunk's queue has been taken
    if (threadIdx.x == 0) Qn = 0;
    __syncthreads();
    const int64_t v = base + threadIdx.x;
    if ((int)threadIdx.x < chunk && v < n && doff[v + 1] - doff[v] > kK4BitsMax) Q[atomicAdd(&Qn, 1)] = (int32_t)v;
    __syncthreads();
    const int32_t nq = Qn;
    for (int32_t qi = 0; qi < nq; ++qi) {  // block-uniform
      const int32_t u = Q[qi];
      const int64_t ub = doff[u];
      const int32_t d = (int32_t)(doff[u + 1] - ub);
      const int32_t P = 1 << (32 - __builtin_clz((uint32_t)(d - 1)));  // power of two >= d, <= CAP
      __syncthreads();  // L of the previous node is no longer read
      for (int32_t i = threadIdx.x; i < P; i += kK4NT) L[i] = i < d ? dcol[ub + i] : kPad;
      __syncthreads();
      for (int32_t i = wv; i < d; i += kK4Waves) acc += wave_k4_pair(L, P, L[i], Cl[wv], doff, dcol, lane);
    }
  }
  k4_block_total<kK4Waves>(acc, reinterpret_cast<unsigned long long*>(L), total);  // L is free after the barrier
}

__global__ void k_zero_one(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0ull;
}

}  // namespace

// Chunk of ids per scan step: enough chunks to fill `target` blocks, at
// most `nt` ids (one per thread).
static int32_t k4_chunk(int32_t n, int64_t target, int32_t nt) {
  const int64_t c = ((int64_t)n + target - 1) / target;
  return (int32_t)(c < 1 ? 1 : c > nt ? nt : c);
}

static unsigned k4_grid(int32_t n, int32_t chunk, int64_t cap) {
  const int64_t g = ((int64_t)n + chunk - 1) / chunk;
  return (unsigned)(g < cap ? g : cap);
}

hipError_t launch_count_k4(int32_t n, const int64_t* doff, const int32_t* dcol, unsigned long long* total,
                           hipStream_t s) {
  k_zero_one<<<1, 64, 0, s>>>(total);
  if (n > 0) {
    const int32_t cm = k4_chunk(n, 65536, kK4NT);
    k_count_k4_bits<0, kK4BitsMid, kK4NT, true><<<k4_grid(n, cm, 65536), kK4NT, 0, s>>>(n, cm, doff, dcol, total);
    const int32_t cb = k4_chunk(n, 1024, 1024);
    k_count_k4_bits<kK4BitsMid, kK4BitsMax, 1024, false><<<k4_grid(n, cb, 1024), 1024, 0, s>>>(n, cb, doff, dcol,
                                                                                                 total);
    k_count_k4<kK4Cap><<<k4_grid(n, cm, 65536), kK4NT, 0, s>>>(n, cm, doff, dcol, total);
  }
  return hipGetLastError();
}

}  // namespace tricc

// 4- and 5-clique counts (clique detection, among the graph-motif methods of
// Section 4): the triangle method one and two sizes up on the same
// degree-ordered DAG. A 4-clique u < w < x < z (by rank) is met once, at u:
// w in N+(u), x in C = N+(u) ∩ N+(w), z in N+(x) ∩ C; a 5-clique adds one
// more level of the same intersection.
#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

constexpr int kK4NT = 256;
// Out-degrees up to kK4BitsMid take the bit-row kernel with 256 threads and
// 39 KB of LDS; up to kK4BitsMax the one with 1,024 threads and 136 KB (one
// block per CU); up to 2,048 the pass kernel over quarters of the positions
// (1,024 threads, 142 KB); up to 4,096 the pass kernel over sixteenths
// (150 KB); up to kK4Cap = 8,192 the pass kernel over blocks of 64
// positions (2 words per row, 102 KB).
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

// Nodes with DMIN < d+(u) <= CAP: bit rows over blocks of PCOLS positions.
// Full rows (up to CAP / 32 words for CAP rows) do not fit in LDS, so the
// block of 1,024 threads makes one pass per PCOLS positions: it builds that
// block of every row (PCOLS / 32 words per row, 128 KB for CAP rows); then
// each wavefront streams N+(w) again, places its ids in N+(u), and for every
// x found (the hits of 64 ids, 64 / (PCOLS / 32) x at a time) adds
// popcount(row w & row x) over the block. Summed over the passes this is the
// count the full rows give. Nodes are queued from chunks of ids as in the
// bit-row kernel.
constexpr int kK4QNT = 1024;
constexpr int kK4QWaves = kK4QNT / kWave;

template <int DMIN, int CAP, int PCOLS>
__global__ __launch_bounds__(kK4QNT) void k_count_k4_passes(int32_t n, int32_t chunk,
                                                            const int64_t* __restrict__ doff,
                                                            const int32_t* __restrict__ dcol,
                                                            unsigned long long* __restrict__ total) {
  constexpr int kK4QCols = PCOLS;
  constexpr int kK4QWords = PCOLS / 32;
  static_assert(PCOLS % 32 == 0 && kK4QWords <= kWave && CAP <= 65536, "pass layout");
  __shared__ int32_t L[CAP];
  __shared__ uint32_t B[CAP * kK4QWords];
  __shared__ uint16_t H[kK4QWaves][kWave];
  __shared__ unsigned long long red[kK4QWaves];
  __shared__ int32_t Q[kK4QNT];
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
      const int64_t dv = doff[v + 1] - doff[v];
      if (dv > DMIN && dv <= CAP) Q[atomicAdd(&Qn, 1)] = (int32_t)v;
    }
    __syncthreads();
    const int32_t nq = Qn;
    for (int32_t qi = 0; qi < nq; ++qi) {  // block-uniform
      const int32_t u = Q[qi];
      const int64_t ub = doff[u];
      const int32_t d = (int32_t)(doff[u + 1] - ub);
      const int32_t P = 1 << (32 - __builtin_clz((uint32_t)(d - 1)));  // power of two >= d, <= CAP
      __syncthreads();  // L and B of the previous node are no longer read
      for (int32_t i = threadIdx.x; i < P; i += kK4QNT) L[i] = i < d ? dcol[ub + i] : kPad;
      for (int32_t q = 0; q * kK4QCols < d; ++q) {
        __syncthreads();  // L written; the previous quarter's rows no longer read
        for (int32_t e = threadIdx.x; e < d * kK4QWords; e += kK4QNT) B[e] = 0u;
        __syncthreads();
        for (int32_t i = wv; i < d; i += kK4QWaves) {  // quarter q of row i
          const int32_t w = L[i];
          const int64_t wb = doff[w];
          const int32_t dw = (int32_t)(doff[w + 1] - wb);
          for (int32_t t = lane; t < dw; t += kWave) {
            const int32_t y = dcol[wb + t];
            const int32_t p = pow2_lower_pos(L, P, y);
            if (L[p] == y && p / kK4QCols == q)
              atomicOr(&B[i * kK4QWords + (p % kK4QCols) / 32], 1u << (p & 31));
          }
        }
        __syncthreads();
        const int32_t k = lane & (kK4QWords - 1);
        const int32_t j = lane / kK4QWords;
        for (int32_t i = wv; i < d; i += kK4QWaves) {  // the x of row i, quarter q of the AND
          const int32_t w = L[i];
          const int64_t wb = doff[w];
          const int32_t dw = (int32_t)(doff[w + 1] - wb);
          const uint32_t bw = B[i * kK4QWords + k];
          for (int32_t t0 = 0; t0 < dw; t0 += kWave) {
            const int32_t t = t0 + lane;
            bool hit = false;
            int32_t p = 0;
            if (t < dw) {
              const int32_t y = dcol[wb + t];
              p = pow2_lower_pos(L, P, y);
              hit = L[p] == y;
            }
            const uint64_t m = __ballot(hit);
            const int32_t nh = (int32_t)__popcll(m);
            if (hit) H[wv][mask_below(m)] = (uint16_t)p;
            wave_sync();
            for (int32_t g = 0; g < nh; g += kWave / kK4QWords) {
              const int32_t jj = g + j;
              if (jj < nh) acc += (unsigned long long)__popc(bw & B[(int32_t)H[wv][jj] * kK4QWords + k]);
            }
            wave_sync();  // H is rewritten by the next 64 ids
          }
        }
      }
    }
  }
  k4_block_total<kK4QWaves>(acc, red, total);
}

// 5-cliques, nodes with DMIN < d+(u) <= DMAX (and d+(u) >= 4): the bit rows
// of the subgraph induced on N+(u) are built as for the 4-clique kernel; a
// 5-clique u < w < x < y < z is then w's row bit x, y a bit of the AND of
// rows w and x, and z a bit of that AND with row y. Each wavefront takes rows
// w in turn and walks the x of row w one at a time: every lane forms one
// word of the AND of rows w and x (lane & (RS - 1)), the y in it are listed
// in LDS (per lane, in bit order, after a scan of the lanes' popcounts), and
// groups of 64 / RS lanes add popcount(AND & row y), one word each.
template <int DMIN, int DMAX, int NT>
__global__ __launch_bounds__(NT) void k_count_k5_bits(int32_t n, int32_t chunk, const int64_t* __restrict__ doff,
                                                      const int32_t* __restrict__ dcol,
                                                      unsigned long long* __restrict__ total) {
  constexpr int NW = NT / kWave;
  static_assert(DMAX % 32 == 0 && DMAX <= 1024, "rows of at most 32 words");
  __shared__ int32_t L[DMAX];
  __shared__ uint32_t B[DMAX * (DMAX / 32)];
  __shared__ uint16_t Y[NW][DMAX];
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
      if (dv >= 4 && dv > DMIN && dv <= DMAX) Q[atomicAdd(&Qn, 1)] = (int32_t)v;
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
      const int32_t k = lane & (RS - 1);
      const int32_t js = lane >> rs;
      for (int32_t i = wv; i < d; i += NW) {
        const uint32_t* Bi = B + i * RS;
        const uint32_t bik = Bi[k];
        for (int32_t kw = 0; kw < RS; ++kw) {
          uint32_t word = Bi[kw];  // wave-uniform
          while (word) {
            const int32_t x = kw * 32 + __builtin_ctz(word);
            word &= word - 1u;
            const uint32_t wx = bik & B[x * RS + k];
            // list the y of wx: lanes 0 .. RS-1 own one word each
            const int32_t c = lane < RS ? __popc(wx) : 0;
            const int32_t incl = wave_incl_scan(c);
            const int32_t ny = __shfl(incl, kWave - 1, kWave);
            if (ny < 2) continue;  // y and z both lie in wx (wave-uniform)
            if (lane < RS) {
              uint32_t bits = wx;
              int32_t o = incl - c;
              while (bits) {
                Y[wv][o++] = (uint16_t)(lane * 32 + __builtin_ctz(bits));
                bits &= bits - 1u;
              }
            }
            wave_sync();
            for (int32_t g = 0; g < ny; g += (kWave >> rs)) {
              const int32_t jj = g + js;
              if (jj < ny) acc += (unsigned long long)__popc(wx & B[(int32_t)Y[wv][jj] * RS + k]);
            }
            wave_sync();  // Y is rewritten for the next x
          }
        }
      }
    }
  }
  k4_block_total<NW>(acc, red, total);
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
    k_count_k4_passes<kK4BitsMax, 2048, 512><<<k4_grid(n, cb, 1024), kK4QNT, 0, s>>>(n, cb, doff, dcol, total);
    k_count_k4_passes<2048, 4096, 256><<<k4_grid(n, cb, 1024), kK4QNT, 0, s>>>(n, cb, doff, dcol, total);
    k_count_k4_passes<4096, kK4Cap, 64><<<k4_grid(n, cb, 1024), kK4QNT, 0, s>>>(n, cb, doff, dcol, total);
  }
  return hipGetLastError();
}

hipError_t launch_count_k5(int32_t n, const int64_t* doff, const int32_t* dcol, unsigned long long* total,
                           hipStream_t s) {
  k_zero_one<<<1, 64, 0, s>>>(total);
  if (n > 0) {
    const int32_t cm = k4_chunk(n, 65536, kK4NT);
    k_count_k5_bits<0, kK4BitsMid, kK4NT><<<k4_grid(n, cm, 65536), kK4NT, 0, s>>>(n, cm, doff, dcol, total);
    const int32_t cb = k4_chunk(n, 2048, 512);
    k_count_k5_bits<kK4BitsMid, kK5Cap, 512><<<k4_grid(n, cb, 2048), 512, 0, s>>>(n, cb, doff, dcol, total);
  }
  return hipGetLastError();
}

}  // namespace tricc

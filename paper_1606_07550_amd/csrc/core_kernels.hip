// Core numbers by parallel level-synchronous peeling (k-core analysis,
// among the analytics methods of Section 4; Section 5 names the
// Batagelj-Zaversnik decomposition, which removes nodes in order of their
// current degree). Here every node whose current degree is at most k is
// removed together (core number k), and the removals lower their
// neighbours' current degrees with atomics; a neighbour that falls to k
// joins the next frontier of the same level. Levels with no node are
// skipped: a scan that finds no frontier reports the smallest current
// degree left.
//
// Scans of every node left are made once per window of levels [k, U]: the
// scan at k also lists the nodes left with current degree <= U (the near
// list), and the peels append every node whose current degree falls from
// U + 1 to U. Every node left with current degree <= U is thus on the near
// list, so the levels up to U scan that list alone.
//
// With `order` given, each node also records the round in which it was
// removed (rounds count every frontier, across levels). A node removed in
// round r had current degree <= k then, counting exactly its neighbours
// removed in round r or later, so orienting every edge towards the later
// (round, id) gives out-degrees at most the core number: the degeneracy
// ordering.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

constexpr int kCoreNT = 256;
constexpr int kPeelG = 8;  // lanes per frontier node in the peel

// Rounds launched together by launch_core_peel_batch, the later ones reading
// their frontier size on the device (a round whose frontier is empty does
// nothing), so the host reads the counters back once per batch.
constexpr int kPeelBatch = 4;
constexpr int64_t kPeelBatchMinNodes = 1024;

// Appends the items of the lanes with `take` to q[*cnt ..], one atomic per
// wavefront. All lanes of the wavefront must call it.
__device__ __forceinline__ void wave_push(bool take, int32_t item, int32_t* __restrict__ q, int32_t* __restrict__ cnt) {
  const uint64_t m = __ballot(take);
  if (!m) return;
  const int leader = __builtin_ctzll(m);
  int32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(cnt, (int32_t)__popcll(m));
  base = __shfl(base, leader, kWave);
  if (take) q[base + mask_below(m)] = item;
}

__global__ __launch_bounds__(kCoreNT) void k_core_init(int32_t n, const int32_t* __restrict__ deg,
                                                       int32_t* __restrict__ cur, int32_t* __restrict__ core) {
  const int64_t stride = (int64_t)gridDim.x * kCoreNT;
  for (int64_t v = (int64_t)blockIdx.x * kCoreNT + threadIdx.x; v < n; v += stride) {
    cur[v] = deg[v];
    core[v] = -1;
  }
}

// cnt[0] = frontier size, cnt[1] = next frontier size, cnt[2] = smallest
// current degree above k among the nodes scanned, cnt[3] = survivors
// listed, cnt[6] and cnt[7] = lengths of the two near-list buffers.
__global__ void k_core_reset(int32_t* __restrict__ cnt, int which, int near) {
  if (which == 2) {  // the speculative rounds' next-frontier counters
    if (threadIdx.x < kPeelBatch) cnt[16 + threadIdx.x] = 0;
    return;
  }
  if (threadIdx.x == 0) {
    if (which == 0) {
      cnt[0] = 0;
      cnt[2] = 0x7fffffff;
      cnt[3] = 0;
    } else {
      cnt[1] = 0;
    }
    if (near >= 0) cnt[near] = 0;
  }
}

// Frontier of level k: the nodes left whose current degree is <= k, among
// the listed candidates A[0, na) (A == NULL: all ids 0 .. na-1). The other
// nodes still left are listed in S (S == NULL: not listed), so later scans
// only visit them.
__global__ __launch_bounds__(kCoreNT) void k_core_scan(int32_t na, const int32_t* __restrict__ A, int32_t k,
                                                       const int32_t* __restrict__ cur, int32_t* __restrict__ core,
                                                       int32_t* __restrict__ F, int32_t* __restrict__ S,
                                                       int32_t* __restrict__ cnt, int32_t* __restrict__ order,
                                                       int32_t round, int32_t U, int32_t* __restrict__ Nr,
                                                       int32_t* __restrict__ ncnt) {
  const int64_t stride = (int64_t)gridDim.x * kCoreNT;
  int32_t mn = 0x7fffffff;
  for (int64_t b = (int64_t)blockIdx.x * kCoreNT; b < na; b += stride) {  // uniform trip count
    const int64_t i = b + threadIdx.x;
    bool take = false, keep = false, near = false;
    int32_t v = 0;
    if (i < na) {
      v = A ? A[i] : (int32_t)i;
      if (core[v] < 0) {
        const int32_t c = cur[v];
        if (c <= k) {
          core[v] = k;
          if (order) order[v] = round;
          take = true;
        } else {
          mn = min(mn, c);
          keep = true;
          near = c <= U;
        }
      }
    }
    wave_push(take, v, F, cnt);
    if (S) wave_push(keep, v, S, cnt + 3);
    if (Nr) wave_push(near, v, Nr, ncnt);
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) mn = min(mn, __shfl_xor(mn, o, kWave));
  if (lane_id() == 0 && mn != 0x7fffffff) atomicMin(cnt + 2, mn);
}

// Rows up to this length are walked by their node's 8-lane group; longer
// ones by the whole wavefront, one node after the other.
constexpr int32_t kPeelShort = 64;
// Steps of a walk issued together: their loads and atomic subtractions are
// in flight at once, since each waits on a round trip to memory.
constexpr int kPeelU = 8;

// kPeelU steps of a walk over row[0, d): the entries j0 + q * W + t, q <
// kPeelU (t = the lane's place among the W walkers). Every lane of the
// wavefront calls it (the pushes are wave-wide).
__device__ __forceinline__ void peel_steps(const int32_t* __restrict__ row, int32_t d, int32_t j0, int32_t W,
                                           int32_t t, int32_t k, int32_t U, int32_t* __restrict__ cur,
                                           int32_t* __restrict__ core, int32_t* __restrict__ order,
                                           int32_t next_round, int32_t* __restrict__ G, int32_t* __restrict__ gcnt,
                                           int32_t* __restrict__ Nr, int32_t* __restrict__ ncnt) {
  int32_t w[kPeelU];
  bool live[kPeelU];
#pragma unroll
  for (int q = 0; q < kPeelU; ++q) {
    const int32_t j = j0 + q * W + t;
    live[q] = j < d;
    w[q] = live[q] ? row[j] : 0;
  }
#pragma unroll
  for (int q = 0; q < kPeelU; ++q) live[q] = live[q] && core[w[q]] < 0;
  int32_t old[kPeelU];
#pragma unroll
  for (int q = 0; q < kPeelU; ++q) old[q] = live[q] ? atomicSub(&cur[w[q]], 1) : 0;
#pragma unroll
  for (int q = 0; q < kPeelU; ++q) {
    // the one decrement from k + 1 to k gives w core number k; the one from
    // U + 1 to U puts it on the near list
    const bool take = live[q] && old[q] == k + 1;
    const bool enter = live[q] && old[q] == U + 1;
    if (take) {
      core[w[q]] = k;
      if (order) order[w[q]] = next_round;
    }
    wave_push(take, w[q], G, gcnt);
    if (Nr) wave_push(enter, w[q], Nr, ncnt);
  }
}

// Removes the frontier F[0, nf) of level k: every neighbour w still left
// loses one from its current degree; the one decrement that takes it from
// k + 1 to k gives it core number k and puts it on the next frontier G.
// nf_dev (may be null): the frontier size is read there (the previous
// round's next-frontier count), not taken from nf; gcnt counts the next
// frontier.
__global__ __launch_bounds__(kCoreNT) void k_core_peel(const int32_t* __restrict__ F, int32_t nf,
                                                       const int32_t* __restrict__ nf_dev, int32_t k,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ deg,
                                                       const int32_t* __restrict__ adj, int32_t* __restrict__ cur,
                                                       int32_t* __restrict__ core, int32_t* __restrict__ G,
                                                       int32_t* __restrict__ gcnt, int32_t* __restrict__ order,
                                                       int32_t round, int32_t U, int32_t* __restrict__ Nr,
                                                       int32_t* __restrict__ ncnt) {
  if (nf_dev) nf = *nf_dev;
  constexpr int GPB = kCoreNT / kPeelG;
  const int lane = lane_id();
  const int g = threadIdx.x % kPeelG;
  const int64_t step = (int64_t)gridDim.x * GPB;
  for (int64_t b = (int64_t)blockIdx.x * GPB; b < nf; b += step) {  // uniform trip count
    const int64_t fi = b + threadIdx.x / kPeelG;
    int32_t dv = 0;
    int64_t rb = 0;
    if (fi < nf) {
      const int32_t v = F[fi];
      dv = deg[v];
      rb = off[v];
    }
    // short rows: each group walks its own, the wavefront its longest short one
    const int32_t ds = dv <= kPeelShort ? dv : 0;
    int32_t dmax = ds;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) dmax = max(dmax, __shfl_xor(dmax, o, kWave));
    for (int32_t j0 = 0; j0 < dmax; j0 += kPeelG * kPeelU)
      peel_steps(adj + rb, ds, j0, kPeelG, g, k, U, cur, core, order, round + 1, G, gcnt, Nr, ncnt);
    // long rows: the whole wavefront on each in turn (group leaders' bits)
    uint64_t longs = __ballot(g == 0 && dv > kPeelShort);
    while (longs) {
      const int src = __builtin_ctzll(longs);
      longs &= longs - 1;
      const int32_t d = __shfl(dv, src, kWave);
      const int64_t r = ((int64_t)__shfl((int32_t)(rb >> 32), src, kWave) << 32) |
                        (uint32_t)__shfl((int32_t)rb, src, kWave);
      for (int32_t j0 = 0; j0 < d; j0 += kWave * kPeelU)
        peel_steps(adj + r, d, j0, kWave, lane, k, U, cur, core, order, round + 1, G, gcnt, Nr, ncnt);
    }
  }
}

__global__ __launch_bounds__(kCoreNT) void k_core_fill(int32_t n, int32_t k, int32_t* __restrict__ core) {
  const int64_t stride = (int64_t)gridDim.x * kCoreNT;
  for (int64_t v = (int64_t)blockIdx.x * kCoreNT + threadIdx.x; v < n; v += stride)
    if (core[v] < 0) core[v] = k;
}

unsigned core_grid(int64_t work) {
  int64_t b = (work + kCoreNT - 1) / kCoreNT;
  return (unsigned)(b < 1 ? 1 : b > 8192 ? 8192 : b);
}

}  // namespace

hipError_t launch_core_init(int32_t n, const int32_t* deg, int32_t* cur, int32_t* core, hipStream_t s) {
  k_core_init<<<core_grid(n), kCoreNT, 0, s>>>(n, deg, cur, core);
  return hipGetLastError();
}

hipError_t launch_core_reset(int32_t* cnt, int which, int near, hipStream_t s) {
  k_core_reset<<<1, 64, 0, s>>>(cnt, which, near);
  return hipGetLastError();
}

hipError_t launch_core_scan(int32_t na, const int32_t* A, int32_t k, const int32_t* cur, int32_t* core, int32_t* F,
                            int32_t* S, int32_t* cnt, int32_t* order, int32_t round, int32_t U, int32_t* Nr,
                            int32_t* ncnt, hipStream_t s) {
  if (na <= 0) return hipSuccess;
  k_core_scan<<<core_grid(na), kCoreNT, 0, s>>>(na, A, k, cur, core, F, S, cnt, order, round, U, Nr, ncnt);
  return hipGetLastError();
}

hipError_t launch_core_peel(const int32_t* F, int32_t nf, int32_t k, const int64_t* off, const int32_t* deg,
                            const int32_t* adj, int32_t* cur, int32_t* core, int32_t* G, int32_t* cnt, int32_t* order,
                            int32_t round, int32_t U, int32_t* Nr, int32_t* ncnt, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  k_core_peel<<<core_grid((int64_t)nf * kPeelG), kCoreNT, 0, s>>>(F, nf, nullptr, k, off, deg, adj, cur, core, G,
                                                                  cnt + 1, order, round, U, Nr, ncnt);
  return hipGetLastError();
}

int core_peel_batch() { return kPeelBatch; }

hipError_t launch_core_peel_batch(int32_t* B0, int32_t* B1, int32_t nf, int32_t k, const int64_t* off,
                                  const int32_t* deg, const int32_t* adj, int32_t* cur, int32_t* core, int32_t* cnt,
                                  int32_t* order, int32_t round, int32_t U, int32_t* Nr, int32_t* ncnt,
                                  hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  k_core_reset<<<1, 64, 0, s>>>(cnt, 2, -1);
  // later rounds read their size on the device; their grid follows the
  // first round's (grid-stride loops take larger frontiers)
  const unsigned grid = core_grid(std::max<int64_t>((int64_t)nf, kPeelBatchMinNodes) * kPeelG);
  for (int i = 0; i < kPeelBatch; ++i)
    k_core_peel<<<grid, kCoreNT, 0, s>>>((i & 1) ? B1 : B0, nf, i ? cnt + 16 + i - 1 : nullptr, k, off, deg, adj,
                                         cur, core, (i & 1) ? B0 : B1, cnt + 16 + i, order, round + i, U, Nr, ncnt);
  return hipGetLastError();
}

hipError_t launch_core_fill(int32_t n, int32_t k, int32_t* core, hipStream_t s) {
  k_core_fill<<<core_grid(n), kCoreNT, 0, s>>>(n, k, core);
  return hipGetLastError();
}

}  // namespace tricc

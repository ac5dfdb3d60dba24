// CSR builder for gfx950: validate + symmetrise + drop self loops (degree
// count, prefix sum, scatter), a segmented row sort binned by row length
// with in-place dedup, and the degree-order orientation into a DAG.
//
// The paper keeps, per node, a vector of adjacent nodes held in sorted order
// (Section 5.1); an undirected edge is stored in both endpoints' vectors.
// Here all vectors live in one array: row v occupies adj[off[v], off[v+1])
// of which the first deg[v] entries are the sorted, duplicate-free
// neighbours once the build is done.
#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

}  // namespace

// ---------------------------------------------------------------------------
// a1: validation and raw degree count (both directions, loops dropped)
__global__ __launch_bounds__(256) void k_degree_raw(const int32_t* __restrict__ src,
                                                    const int32_t* __restrict__ dst, int64_t m_raw,
                                                    int32_t n, int32_t* __restrict__ cnt,
                                                    int32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m_raw; e += stride) {
    const int32_t u = src[e], v = dst[e];
    if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n) { bad = true; continue; }
    if (u == v) continue;
    atomicAdd(&cnt[u], 1);
    atomicAdd(&cnt[v], 1);
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(err, 1);
}

hipError_t launch_degree_raw(const int32_t* src, const int32_t* dst, int64_t m_raw, int32_t n,
                             int32_t* cnt, int32_t* err, hipStream_t s) {
  if (m_raw == 0) return hipSuccess;
  k_degree_raw<<<grid_for(m_raw, 256 * 8, 1u << 16), 256, 0, s>>>(src, dst, m_raw, n, cnt, err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum (reduce, scan of block sums, apply).
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int64_t kScanTile = kScanThreads * kScanItems;

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

template <typename Tin>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const Tin* __restrict__ in, int64_t n,
                                                              int64_t* __restrict__ bsum) {
  __shared__ int64_t lds[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) acc += (int64_t)in[i];
  }
  const int64_t t = block_sum<int64_t, kScanThreads>(acc, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// Single block: exclusive scan of nb block sums in place; bsum[nb] = total.
__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ int64_t lds[1024 / kWave + 1];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t x = i < nb ? bsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<int64_t, 1024>(x, lds, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

template <typename Tin>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const Tin* __restrict__ in, int64_t n,
                                                             const int64_t* __restrict__ bsum,
                                                             int64_t* __restrict__ out, int64_t nb) {
  __shared__ int64_t lds[kScanThreads / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  // blocked arrangement: thread t owns kScanItems consecutive elements
  int64_t v[kScanItems];
  int64_t acc = 0;
  const int64_t tb = base + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = tb + k;
    v[k] = i < n ? (int64_t)in[i] : 0;
    acc += v[k];
  }
  int64_t tot;
  int64_t run = bsum[blockIdx.x] + block_excl_scan<int64_t, kScanThreads>(acc, lds, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = tb + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

template <typename Tin>
static hipError_t scan_impl(const Tin* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    return hipMemsetAsync(out, 0, sizeof(int64_t), s);
  }
  k_scan_reduce<Tin><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, tmp);
  k_scan_blocks<<<1, 1024, 0, s>>>(tmp, nb);
  k_scan_apply<Tin><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, tmp, out, nb);
  return hipGetLastError();
}

hipError_t launch_scan_i32(const int32_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
  return scan_impl<int32_t>(in, n, out, tmp, s);
}
hipError_t launch_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
  return scan_impl<int64_t>(in, n, out, tmp, s);
}

// ---------------------------------------------------------------------------
// a1/a3: scatter both directions into the row segments (unsorted).
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ dst, int64_t m_raw,
                                                 const int64_t* __restrict__ off,
                                                 int32_t* __restrict__ cur, int32_t* __restrict__ adj) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m_raw; e += stride) {
    const int32_t u = src[e], v = dst[e];
    if (u == v) continue;
    adj[off[u] + atomicAdd(&cur[u], 1)] = v;
    adj[off[v] + atomicAdd(&cur[v], 1)] = u;
  }
}

hipError_t launch_scatter(const int32_t* src, const int32_t* dst, int64_t m_raw, const int64_t* off,
                          int32_t* cur, int32_t* adj, hipStream_t s) {
  if (m_raw == 0) return hipSuccess;
  k_scatter<<<grid_for(m_raw, 256 * 8, 1u << 16), 256, 0, s>>>(src, dst, m_raw, off, cur, adj);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a1-a3, partitioned: the same raw rows without a global atomic per entry.
// Node v lies in partition v >> pbits (2^pbits consecutive ids, at most
// kPartMax partitions). Pass A counts each partition's entries with LDS
// histograms (and checks the ids); pass B moves every entry, i.e. each pair
// seen from each of its endpoints, into its partition's slice of a staging
// array (other endpoint in pv, the row as a 16-bit local index in pu),
// reserving one range per (tile, partition); passes C and D take one chunk
// of one partition per block with one LDS counter per node of the
// partition: C adds up the raw row lengths, D reserves each row's range and
// places the entries. Self loops are dropped in A and B.
constexpr int kPartMax = kPartMaxParts;
constexpr int kPartMinBits = 10, kPartMaxBits = 14;
constexpr int kPartNT = 1024;
constexpr int kPartPairs = 16;  // pairs per thread per tile in pass B
constexpr int64_t kPartTile = (int64_t)kPartNT * kPartPairs;
constexpr int kRowsNT = 1024;
constexpr int kRowsUnroll = 2;  // groups of 8 entries per thread per step
constexpr int64_t kRowsChunk = int64_t(1) << 18;  // entries per block in C and D

int part_bits(int64_t n) {
  if (n <= 0) return -1;
  int b = kPartMinBits;
  while (b < kPartMaxBits && ((n + (int64_t(1) << b) - 1) >> b) > 1024) ++b;
  return ((n + (int64_t(1) << b) - 1) >> b) <= kPartMax ? b : -1;
}

__global__ __launch_bounds__(kPartNT) void k_part_count(const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ dst, int64_t m_raw, int32_t n,
                                                       int pbits, int32_t P, uint32_t* __restrict__ ptotal,
                                                       int32_t* __restrict__ err) {
  __shared__ uint32_t hist[kPartMax];
  for (int b = threadIdx.x; b < P; b += kPartNT) hist[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kPartNT;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * kPartNT + threadIdx.x; e < m_raw; e += stride) {
    const int32_t u = src[e], v = dst[e];
    if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n) { bad = true; continue; }
    if (u == v) continue;
    atomicAdd(&hist[u >> pbits], 1u);
    atomicAdd(&hist[v >> pbits], 1u);
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(err, 1);
  __syncthreads();
  for (int b = threadIdx.x; b < P; b += kPartNT)
    if (hist[b]) atomicAdd(&ptotal[b], hist[b]);
}

// Single block: pstart = exclusive scan of the partition sizes, cstart =
// exclusive scan of their chunk counts (ceil(size / kRowsChunk)).
__global__ __launch_bounds__(1024) void k_part_scan(const uint32_t* __restrict__ ptotal, int32_t P,
                                                    int64_t* __restrict__ pstart, int64_t* __restrict__ cstart) {
  __shared__ int64_t lds[1024 / kWave + 1];
  int64_t c0 = 0, c1 = 0;
  for (int32_t base = 0; base < P; base += 1024) {
    const int32_t i = base + threadIdx.x;
    const int64_t t = i < P ? (int64_t)ptotal[i] : 0;
    const int64_t ch = (t + kRowsChunk - 1) / kRowsChunk;
    int64_t tot0, tot1;
    const int64_t e0 = block_excl_scan<int64_t, 1024>(t, lds, &tot0);
    const int64_t e1 = block_excl_scan<int64_t, 1024>(ch, lds, &tot1);
    if (i < P) {
      pstart[i] = c0 + e0;
      cstart[i] = c1 + e1;
    }
    c0 += tot0;
    c1 += tot1;
  }
  if (threadIdx.x == 0) {
    pstart[P] = c0;
    cstart[P] = c1;
  }
}

// Pass B: ids are known to be in range (pass A checked them).
__global__ __launch_bounds__(kPartNT) void k_part_place(const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ dst, int64_t m_raw, int pbits,
                                                       int32_t P, const int64_t* __restrict__ pstart,
                                                       uint32_t* __restrict__ pcur, int32_t* __restrict__ pv,
                                                       uint16_t* __restrict__ pu) {
  __shared__ uint32_t hist[kPartMax];
  __shared__ int64_t hoff[kPartMax];
  const int64_t ntiles = (m_raw + kPartTile - 1) / kPartTile;
  const int32_t lmask = (1 << pbits) - 1;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int b = threadIdx.x; b < P; b += kPartNT) hist[b] = 0;
    __syncthreads();
    const int64_t base = tile * kPartTile + threadIdx.x;
    int32_t a[kPartPairs], c[kPartPairs];
#pragma unroll
    for (int k = 0; k < kPartPairs; ++k) {
      const int64_t e = base + (int64_t)k * kPartNT;
      a[k] = -1;
      c[k] = -1;
      if (e < m_raw) {
        a[k] = src[e];
        c[k] = dst[e];
      }
    }
    uint32_t ra[kPartPairs], rc[kPartPairs];
#pragma unroll
    for (int k = 0; k < kPartPairs; ++k) {
      if (a[k] == c[k]) a[k] = -1;  // self loop or past the end
      if (a[k] >= 0) {
        ra[k] = atomicAdd(&hist[a[k] >> pbits], 1u);
        rc[k] = atomicAdd(&hist[c[k] >> pbits], 1u);
      }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < P; b += kPartNT) {
      const uint32_t h = hist[b];
      if (h) hoff[b] = pstart[b] + atomicAdd(&pcur[b], h);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPartPairs; ++k) {
      if (a[k] < 0) continue;
      const int64_t p = hoff[a[k] >> pbits] + ra[k];
      pv[p] = c[k];
      pu[p] = (uint16_t)(a[k] & lmask);
      const int64_t q = hoff[c[k] >> pbits] + rc[k];
      pv[q] = a[k];
      pu[q] = (uint16_t)(c[k] & lmask);
    }
    __syncthreads();  // hist and hoff are reused by the next tile
  }
}

// Pass B with coalesced stores, for at most kStagedParts partitions: a tile
// of kStagedPairs pairs is ranked per partition (LDS atomics), scanned, and
// staged in LDS in partition order; each partition's run then goes to its
// reserved range with consecutive lanes on consecutive addresses, instead
// of one cache line per lane.
constexpr int kStagedParts = 1024;
constexpr int kStagedNT = 1024;
constexpr int kStagedPairs = 8192;
constexpr int kStagedPer = kStagedPairs / kStagedNT;

__global__ __launch_bounds__(kStagedNT) void k_part_place_staged(const int32_t* __restrict__ src,
                                                                 const int32_t* __restrict__ dst, int64_t m_raw,
                                                                 int pbits, int32_t P,
                                                                 const int64_t* __restrict__ pstart,
                                                                 uint32_t* __restrict__ pcur, int32_t* __restrict__ pv,
                                                                 uint16_t* __restrict__ pu) {
  __shared__ uint32_t cnt[kStagedParts];   // entries of each partition in the tile
  __shared__ uint32_t lst[kStagedParts];   // their exclusive prefix (run start in the stage)
  __shared__ int64_t hoff[kStagedParts];   // global start of the run
  __shared__ int32_t sv[2 * kStagedPairs];  // staged other endpoint
  __shared__ int32_t ss[2 * kStagedPairs];  // staged row endpoint
  __shared__ uint32_t red[kStagedNT / kWave + 1];
  const int64_t ntiles = (m_raw + kStagedPairs - 1) / kStagedPairs;
  const int32_t lmask = (1 << pbits) - 1;
  constexpr int BPT = kStagedParts / kStagedNT;  // bins per thread in the scan
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int b = threadIdx.x; b < P; b += kStagedNT) cnt[b] = 0;
    __syncthreads();
    int32_t a[kStagedPer], c[kStagedPer];
    uint32_t ra[kStagedPer], rc[kStagedPer];
    const int64_t base = tile * kStagedPairs + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kStagedPer; ++k) {
      const int64_t e = base + (int64_t)k * kStagedNT;
      a[k] = -1;
      c[k] = -1;
      if (e < m_raw) {
        a[k] = src[e];
        c[k] = dst[e];
      }
    }
#pragma unroll
    for (int k = 0; k < kStagedPer; ++k) {
      if (a[k] == c[k]) a[k] = -1;  // self loop or past the end
      if (a[k] >= 0) {
        ra[k] = atomicAdd(&cnt[a[k] >> pbits], 1u);
        rc[k] = atomicAdd(&cnt[c[k] >> pbits], 1u);
      }
    }
    __syncthreads();
    // exclusive scan of cnt over the partitions (BPT consecutive bins per thread)
    uint32_t loc[BPT > 0 ? BPT : 1];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int b = threadIdx.x * BPT + q;
      loc[q] = b < P ? cnt[b] : 0u;
      sum += loc[q];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<uint32_t, kStagedNT>(sum, red, &tot);
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int b = threadIdx.x * BPT + q;
      if (b < P) {
        lst[b] = run;
        if (loc[q]) hoff[b] = pstart[b] + atomicAdd(&pcur[b], loc[q]);
      }
      run += loc[q];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kStagedPer; ++k) {
      if (a[k] < 0) continue;
      const uint32_t i = lst[a[k] >> pbits] + ra[k];
      sv[i] = c[k];
      ss[i] = a[k];
      const uint32_t j = lst[c[k] >> pbits] + rc[k];
      sv[j] = a[k];
      ss[j] = c[k];
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < tot; t += kStagedNT) {
      const int32_t r = ss[t];
      const int32_t p = r >> pbits;
      const int64_t pos = hoff[p] + (t - lst[p]);
      pv[pos] = sv[t];
      pu[pos] = (uint16_t)(r & lmask);
    }
    __syncthreads();  // the stage and the tables are reused by the next tile
  }
}

// Passes C (pass 0) and D (pass 1). Block c takes chunk c; blocks past the
// last chunk exit. A partition held by one chunk writes its rows directly;
// one spread over several chunks combines them with global atomics (len for
// C, the zeroed cursors cur for D).
__global__ __launch_bounds__(kRowsNT) void k_part_rows(int pass, int pbits, int32_t P, int32_t n,
                                                      const int64_t* __restrict__ pstart,
                                                      const int64_t* __restrict__ cstart,
                                                      const uint16_t* __restrict__ pu,
                                                      const int32_t* __restrict__ pv, int32_t* __restrict__ len,
                                                      const int64_t* __restrict__ raw_off,
                                                      int32_t* __restrict__ cur, int32_t* __restrict__ adj) {
  __shared__ uint32_t cnt[1 << kPartMaxBits];
  const int64_t c = blockIdx.x;
  if (c >= cstart[P]) return;
  // partition of chunk c: the last p with cstart[p] <= c (empty partitions
  // share their start with the next one and are skipped)
  int32_t lo = 0, hi = P - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (cstart[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int32_t p = lo;
  const int64_t pb = pstart[p];
  const int64_t i0 = pb + (c - cstart[p]) * kRowsChunk;
  const int64_t i1 = min(pstart[p + 1], i0 + kRowsChunk);
  const bool single = cstart[p + 1] - cstart[p] == 1;
  const int32_t v0 = p << pbits;
  const int32_t W = min(1 << pbits, n - v0);
  for (int j = threadIdx.x; j < W; j += kRowsNT) cnt[j] = 0;
  __syncthreads();
  // aligned groups of 8 entries, one 16-byte load of local rows each (the
  // group start rounds down inside the array; the last group may read up
  // to 7 entries past the end, inside the staging area's padding); entries
  // outside [i0, i1) are masked
  const int64_t g0 = i0 & ~int64_t(7);
  for (int64_t gs = g0 + 8 * (int64_t)threadIdx.x; gs < i1; gs += 8 * kRowsNT * kRowsUnroll) {
    uint4 w[kRowsUnroll];
#pragma unroll
    for (int k = 0; k < kRowsUnroll; ++k) {
      const int64_t at = gs + (int64_t)k * 8 * kRowsNT;
      w[k] = at < i1 ? *reinterpret_cast<const uint4*>(pu + at) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < kRowsUnroll; ++k) {
      const int64_t at = gs + (int64_t)k * 8 * kRowsNT;
      const uint32_t ws[4] = {w[k].x, w[k].y, w[k].z, w[k].w};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t i = at + q;
        if (i >= i0 && i < i1) atomicAdd(&cnt[(ws[q >> 1] >> (16 * (q & 1))) & 0xffffu], 1u);
      }
    }
  }
  __syncthreads();
  if (pass == 0) {
    for (int j = threadIdx.x; j < W; j += kRowsNT) {
      const uint32_t k = cnt[j];
      if (!k) continue;
      if (single) len[v0 + j] = (int32_t)k;
      else atomicAdd(&len[v0 + j], (int32_t)k);
    }
    return;
  }
  for (int j = threadIdx.x; j < W; j += kRowsNT) {
    const uint32_t k = cnt[j];
    if (!k) continue;
    const int32_t at = single ? 0 : atomicAdd(&cur[v0 + j], (int32_t)k);
    cnt[j] = (uint32_t)(raw_off[v0 + j] - pb) + (uint32_t)at;
  }
  __syncthreads();
  for (int64_t gs = g0 + 8 * (int64_t)threadIdx.x; gs < i1; gs += 8 * kRowsNT * kRowsUnroll) {
    uint4 w[kRowsUnroll];
    int4 xa[kRowsUnroll], xb[kRowsUnroll];
#pragma unroll
    for (int k = 0; k < kRowsUnroll; ++k) {
      const int64_t at = gs + (int64_t)k * 8 * kRowsNT;
      const bool ok = at < i1;
      w[k] = ok ? *reinterpret_cast<const uint4*>(pu + at) : make_uint4(0, 0, 0, 0);
      xa[k] = ok ? *reinterpret_cast<const int4*>(pv + at) : make_int4(0, 0, 0, 0);
      xb[k] = ok ? *reinterpret_cast<const int4*>(pv + at + 4) : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < kRowsUnroll; ++k) {
      const int64_t at = gs + (int64_t)k * 8 * kRowsNT;
      const uint32_t ws[4] = {w[k].x, w[k].y, w[k].z, w[k].w};
      const int32_t xs[8] = {xa[k].x, xa[k].y, xa[k].z, xa[k].w, xb[k].x, xb[k].y, xb[k].z, xb[k].w};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t i = at + q;
        if (i >= i0 && i < i1) adj[pb + atomicAdd(&cnt[(ws[q >> 1] >> (16 * (q & 1))) & 0xffffu], 1u)] = xs[q];
      }
    }
  }
}

hipError_t launch_part_count(const int32_t* src, const int32_t* dst, int64_t m_raw, int32_t n, int pbits, int32_t P,
                             uint32_t* ptotal, int32_t* err, hipStream_t s) {
  if (m_raw == 0) return hipSuccess;
  k_part_count<<<grid_for(m_raw, kPartNT * 16, 2048), kPartNT, 0, s>>>(src, dst, m_raw, n, pbits, P, ptotal, err);
  return hipGetLastError();
}

hipError_t launch_part_scan(const uint32_t* ptotal, int32_t P, int64_t* pstart, int64_t* cstart, hipStream_t s) {
  k_part_scan<<<1, 1024, 0, s>>>(ptotal, P, pstart, cstart);
  return hipGetLastError();
}

hipError_t launch_part_place(const int32_t* src, const int32_t* dst, int64_t m_raw, int pbits, int32_t P,
                             const int64_t* pstart, uint32_t* pcur, int32_t* pv, uint16_t* pu, hipStream_t s) {
  if (m_raw == 0) return hipSuccess;
  if (P <= kStagedParts) {
    k_part_place_staged<<<grid_for(m_raw, kStagedPairs, 4096), kStagedNT, 0, s>>>(src, dst, m_raw, pbits, P, pstart,
                                                                                 pcur, pv, pu);
    return hipGetLastError();
  }
  k_part_place<<<grid_for(m_raw, (int)kPartTile, 4096), kPartNT, 0, s>>>(src, dst, m_raw, pbits, P, pstart, pcur,
                                                                         pv, pu);
  return hipGetLastError();
}

hipError_t launch_part_rows(int pass, int pbits, int32_t P, int32_t n, int64_t max_entries, const int64_t* pstart,
                            const int64_t* cstart, const uint16_t* pu, const int32_t* pv, int32_t* len,
                            const int64_t* raw_off, int32_t* cur, int32_t* adj, hipStream_t s) {
  // every partition has at most ceil(size / chunk) <= size / chunk + 1 chunks
  const int64_t blocks = max_entries / kRowsChunk + P + 1;
  k_part_rows<<<(unsigned)blocks, kRowsNT, 0, s>>>(pass, pbits, P, n, pstart, cstart, pu, pv, len, raw_off, cur, adj);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row classes by raw length.
__device__ __forceinline__ int row_class(int32_t len) {
  if (len <= 1) return kRowTrivial;
  if (len <= 8) return kRow8;
  if (len <= 16) return kRow16;
  if (len <= 32) return kRow32;
  if (len <= 64) return kRow64;
  if (len <= 128) return kRow128;
  if (len <= 256) return kRow256;
  if (len <= 512) return kRow512;
  if (len <= 1024) return kRow1024;
  if (len <= 4096) return kRowLds4k;
  if (len <= 8192) return kRowLds8k;
  if (len <= kLargeChunk) return kRowLds32k;
  return kRowLarge;
}

// Classification of [0, n) into classes with per-block histograms: pass 0
// counts each block's members per class (LDS atomics) into
// hist[c * nblk + blk]; the host scans hist; pass 1 writes each member at
// off[c * nblk + blk] + its rank inside the block. No global atomics.
constexpr int kClsThreads = 256;
constexpr int64_t kClsChunk = 4096;

int64_t classify_blocks(int64_t n) { return (n + kClsChunk - 1) / kClsChunk; }

struct RowClassOf {  // by raw row length; trivial rows are not listed
  const int32_t* len;
  int32_t* deg;
  __device__ int operator()(int64_t v, int pass) const {
    const int32_t L = len[v];
    const int c = row_class(L);
    if (c == kRowTrivial) {
      if (pass == 0) deg[v] = L;
      return -1;
    }
    return c;
  }
};

struct NodeBinOf {  // by DAG out-degree; nodes with d+ < 2 are not listed
  const int32_t* dplus;
  const int32_t* limit;
  __device__ int operator()(int64_t v, int) const {
    const int32_t d = dplus[v];
    if (d < 2) return -1;
    int b = kNumBins - 1;
#pragma unroll
    for (int q = kNumBins - 2; q >= 0; --q)
      if (d <= limit[q]) b = q;
    return b;
  }
};

struct InBinOf {  // in-list pass owners: 3 <= d+(w) <= limit[4], at least one in-neighbour
  const int32_t* dplus;
  const int32_t* deg;
  const int32_t* limit;
  __device__ int operator()(int64_t v, int) const {
    const int32_t d = dplus[v];
    if (d < 3 || deg[v] - d < 1 || d > limit[kNumBins - 2]) return -1;
    int b = kNumBins - 2;
#pragma unroll
    for (int q = kNumBins - 3; q >= 0; --q)
      if (d <= limit[q]) b = q;
    return b;
  }
};

template <int NC, class F>
__global__ __launch_bounds__(kClsThreads) void k_classify(int pass, int64_t n, F f, int32_t* __restrict__ hist,
                                                          const int64_t* __restrict__ off, int64_t nblk,
                                                          int32_t* __restrict__ list) {
  __shared__ int32_t cnt[NC];
  if (threadIdx.x < NC) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kClsChunk;
  const int64_t b1 = min(n, b0 + kClsChunk);
  for (int64_t v = b0 + threadIdx.x; v < b1; v += kClsThreads) {
    const int c = f(v, pass);
    if (c < 0) continue;
    const int32_t r = atomicAdd(&cnt[c], 1);
    if (pass == 1) list[off[(int64_t)c * nblk + blockIdx.x] + r] = (int32_t)v;
  }
  if (pass == 0) {
    __syncthreads();
    if (threadIdx.x < NC) hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
  }
}

__global__ void k_class_offsets(const int64_t* __restrict__ off, int64_t nblk, int nc, int64_t* __restrict__ cls_off) {
  const int c = threadIdx.x;
  if (c <= nc) cls_off[c] = off[(int64_t)c * nblk];
}

hipError_t launch_classify_rows(int pass, int32_t n, const int32_t* len, int32_t* deg, int32_t* hist,
                                const int64_t* off, int64_t nblk, int32_t* list, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_classify<kNumRowClasses, RowClassOf><<<(unsigned)nblk, kClsThreads, 0, s>>>(pass, n, RowClassOf{len, deg}, hist,
                                                                               off, nblk, list);
  return hipGetLastError();
}

hipError_t launch_classify_bins(int pass, int32_t n, const int32_t* dplus, const int32_t* limit, int32_t* hist,
                                const int64_t* off, int64_t nblk, int32_t* list, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_classify<kNumBins, NodeBinOf><<<(unsigned)nblk, kClsThreads, 0, s>>>(pass, n, NodeBinOf{dplus, limit}, hist, off,
                                                                        nblk, list);
  return hipGetLastError();
}

hipError_t launch_classify_inbins(int pass, int32_t n, const int32_t* dplus, const int32_t* deg, const int32_t* limit,
                                  int32_t* hist, const int64_t* off, int64_t nblk, int32_t* list, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_classify<kNumBins, InBinOf><<<(unsigned)nblk, kClsThreads, 0, s>>>(pass, n, InBinOf{dplus, deg, limit}, hist, off,
                                                                      nblk, list);
  return hipGetLastError();
}

__global__ void k_gather_offsets(const int64_t* __restrict__ prefix, const int64_t* __restrict__ at, int k,
                                 int64_t* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) out[i] = prefix[at[i]];
}

hipError_t launch_gather_offsets(const int64_t* prefix, const int64_t* at, int k, int64_t* out, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  k_gather_offsets<<<(unsigned)std::min(1024, (k + 255) / 256), 256, 0, s>>>(prefix, at, k, out);
  return hipGetLastError();
}

hipError_t launch_class_offsets(const int64_t* off, int64_t nblk, int nc, int64_t* cls_off, hipStream_t s) {
  k_class_offsets<<<1, 64, 0, s>>>(off, nblk, nc, cls_off);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ constexpr uint64_t group_bits() {
  return G >= 64 ? ~0ull : ((1ull << (G & 63)) - 1);
}

// Rows of up to G entries: a group of G lanes sorts one row in registers with
// a bitonic network over __shfl_xor, then compacts the unique values.
template <int G>
__global__ __launch_bounds__(256) void k_sort_small(const int32_t* __restrict__ rows, int32_t nrows,
                                                    const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ len,
                                                    int32_t* __restrict__ adj, int32_t* __restrict__ deg) {
  const int gi = (blockIdx.x * 256 + threadIdx.x) / G;
  const int g = threadIdx.x % G;
  const bool active = gi < nrows;
  int32_t v = 0, L = 0;
  int64_t beg = 0;
  int32_t x = kPad;
  if (active) {
    v = rows[gi];
    beg = off[v];
    L = len[v];
    if (g < L) x = adj[beg + g];
  }
#pragma unroll
  for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int32_t y = __shfl_xor(x, j, G);
      const bool up = (g & k) == 0;
      const bool low = (g & j) == 0;
      x = (low == up) ? min(x, y) : max(x, y);
    }
  }
  const int32_t prev = __shfl_up(x, 1, G);
  const bool uniq = active && x != kPad && (g == 0 || x != prev);
  const uint64_t mask = __ballot(uniq);
  const int shift = lane_id() & ~(G - 1);
  const uint64_t gm = (mask >> shift) & group_bits<G>();
  if (uniq) adj[beg + __popcll(gm & ((1ull << g) - 1))] = x;
  if (active && g == 0) deg[v] = (int32_t)__popcll(gm);
}

// Bitonic compare-exchanges of one stride j of stage k on kSortRun ids held
// by one thread in registers (x[r] is id base + r); run-local strides only.
constexpr int kSortRun = 32;
__device__ __forceinline__ void run_stage(int32_t (&x)[kSortRun], int base, int j, int k) {
#pragma unroll
  for (int r = 0; r < kSortRun; ++r) {
    const int pr = r ^ j;
    if (pr > r) {
      const bool up = ((base + r) & k) == 0;
      const int32_t a = x[r], b = x[pr];
      x[r] = up ? min(a, b) : max(a, b);
      x[pr] = up ? max(a, b) : min(a, b);
    }
  }
}

// Rows of up to CAP entries: one block sorts one row (or one chunk) in LDS
// with a bitonic network. Each thread owns a run of 32 consecutive ids: the
// strides below 32 run in its registers (one LDS read and write for all of
// them, the first five stages in one pass), the larger strides in LDS, one
// barrier each. The LDS holds id i at i + i / 32, so a run's ids sit in
// distinct banks for the 32 lanes that read them together. DEDUP: compact
// the unique values in place and write deg; otherwise write the sorted chunk
// back as is. Rows of at most lmin entries are left to another kernel.
template <int CAP, int NT, bool DEDUP>
__global__ __launch_bounds__(NT) void k_sort_lds(const int32_t* __restrict__ rows,
                                                 const int64_t* __restrict__ seg_beg,
                                                 const int32_t* __restrict__ seg_len,
                                                 const int64_t* __restrict__ off,
                                                 const int32_t* __restrict__ len,
                                                 int32_t* __restrict__ adj, int32_t* __restrict__ deg,
                                                 int32_t lmin) {
  constexpr int R = kSortRun;
  static_assert(CAP % R == 0 && CAP / R <= NT, "one run per thread");
  __shared__ int32_t s[CAP + CAP / R];
  __shared__ int32_t lds_scan[NT / kWave + 1];
  auto at = [](int i) { return i + (i >> 5); };
  int32_t v = -1;
  int64_t beg;
  int32_t L;
  if (DEDUP) {
    v = rows[blockIdx.x];
    beg = off[v];
    L = len[v];
  } else {
    beg = seg_beg[blockIdx.x];
    L = seg_len[blockIdx.x];
  }
  if (L <= lmin) return;  // block-uniform
  int P = R;
  while (P < L) P <<= 1;
  for (int i = threadIdx.x; i < P; i += NT) s[at(i)] = i < L ? adj[beg + i] : kPad;
  __syncthreads();
  const int g = threadIdx.x;
  const bool owner = g < P / R;  // thread g owns ids g R .. g R + R - 1, at g (R + 1) + r
  int32_t x[R];
  if (owner) {
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = s[g * (R + 1) + r];
#pragma unroll
    for (int k = 2; k <= R; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) run_stage(x, g * R, j, k);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) s[g * (R + 1) + r] = x[r];
  }
  __syncthreads();
  for (int k = 2 * R; k <= P; k <<= 1) {
    for (int j = k >> 1; j >= R; j >>= 1) {
      for (int i = threadIdx.x; i < (P >> 1); i += NT) {
        const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const int32_t a = s[at(lo)], b = s[at(hi)];
        if ((a > b) == up) { s[at(lo)] = b; s[at(hi)] = a; }
      }
      __syncthreads();
    }
    if (owner) {
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = s[g * (R + 1) + r];
#pragma unroll
      for (int j = R >> 1; j > 0; j >>= 1) run_stage(x, g * R, j, k);
#pragma unroll
      for (int r = 0; r < R; ++r) s[g * (R + 1) + r] = x[r];
    }
    __syncthreads();
  }
  if (!DEDUP) {
    for (int i = threadIdx.x; i < L; i += NT) adj[beg + i] = s[at(i)];
    return;
  }
  int32_t carry = 0;
  for (int base = 0; base < L; base += NT) {
    const int i = base + threadIdx.x;
    const int32_t x0 = i < L ? s[at(i)] : kPad;
    const bool u = i < L && (i == 0 || x0 != s[at(i - 1)]);
    int32_t tot;
    const int32_t ex = block_excl_scan<int32_t, NT>(u ? 1 : 0, lds_scan, &tot);
    if (u) adj[beg + carry + ex] = x0;
    carry += tot;
  }
  if (threadIdx.x == 0) deg[v] = carry;
}

// Rows of up to 64 * E raw entries: one wavefront per row (grid-stride), the
// row in registers (id i in lane i % 64, register i / 64), a bitonic network
// whose strides >= 64 swap registers inside a lane and whose smaller strides
// exchange with the lane i ^ j by a shuffle, so no LDS and no barrier.
// Then an in-order dedup and a compacted, coalesced write to the row start.
template <int E>
__global__ __launch_bounds__(256) void k_sort_wave(const int32_t* __restrict__ rows, int32_t nrows,
                                                   const int64_t* __restrict__ off, const int32_t* __restrict__ len,
                                                   int32_t* __restrict__ adj, int32_t* __restrict__ deg) {
  constexpr int P = kWave * E;
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * (256 / kWave);
  for (int64_t r = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave; r < nrows; r += nw) {
    const int32_t v = rows[r];
    const int64_t beg = off[v];
    const int32_t L = len[v];
    int32_t x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int32_t i = e * kWave + lane;
      x[e] = i < L ? adj[beg + i] : kPad;
    }
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        if (j >= kWave) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int pe = e ^ (j / kWave);
            if (pe > e) {
              const bool up = ((e * kWave) & k) == 0;  // k > 64: the lane bits do not matter
              const int32_t a = x[e], b = x[pe];
              x[e] = up ? min(a, b) : max(a, b);
              x[pe] = up ? max(a, b) : min(a, b);
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            const int32_t y = __shfl_xor(x[e], j, kWave);
            const bool up = ((e * kWave + lane) & k) == 0;
            const bool lo = (lane & j) == 0;
            x[e] = (lo == up) ? min(x[e], y) : max(x[e], y);
          }
        }
      }
    }
    int32_t base = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int32_t i = e * kWave + lane;
      int32_t prev = __shfl_up(x[e], 1, kWave);
      if (e > 0) {
        const int32_t last = __builtin_amdgcn_readlane(x[e > 0 ? e - 1 : 0], kWave - 1);
        if (lane == 0) prev = last;
      }
      const bool u = i < L && (i == 0 || x[e] != prev);
      const uint64_t m = __ballot(u);
      if (u) adj[beg + base + mask_below(m)] = x[e];
      base += (int32_t)__popcll(m);
    }
    if (lane == 0) deg[v] = base;
  }
}

// Rows (or chunks) of up to 64 * E * W ids: one block of W wavefronts holds
// the row in registers (id i in wavefront i / (64 E), register (i / 64) % E,
// lane i % 64) and runs a bitonic network on it: strides below 64 exchange
// by shuffles, strides below 64 E swap registers inside a lane, and only the
// strides of 64 E and up go through LDS (write, barrier, read of the partner,
// barrier). The stages run in a loop over k with the strides unrolled, which
// keeps the code small. The network spans only the next power of two Q >= L
// (the first Q ids, ascending; the pads beyond are left as they are), and
// wavefronts wholly past Q skip the register and shuffle stages. DEDUP: the
// unique ids, compacted to the row start, and deg[v]; otherwise the sorted
// chunk back in place. Rows longer than the block holds are left alone.
template <int E, int W, bool DEDUP>
__global__ __launch_bounds__(kWave * W) void k_sort_block(const int32_t* __restrict__ rows,
                                                          const int64_t* __restrict__ seg_beg,
                                                          const int32_t* __restrict__ seg_len,
                                                          const int64_t* __restrict__ off,
                                                          const int32_t* __restrict__ len,
                                                          int32_t* __restrict__ adj, int32_t* __restrict__ deg) {
  constexpr int PW = kWave * E;  // ids per wavefront
  constexpr int P = PW * W;
  __shared__ int32_t s[P];
  __shared__ int32_t wsum[W + 1];
  __shared__ int32_t wlast[W];
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const int32_t i0 = wv * PW + lane;  // index of x[0]; x[e] is i0 + 64 e
  int32_t v = -1;
  int64_t beg;
  int32_t L;
  if (DEDUP) {
    v = rows[blockIdx.x];
    beg = off[v];
    L = len[v];
  } else {
    beg = seg_beg[blockIdx.x];
    L = seg_len[blockIdx.x];
  }
  if (L > P) return;  // block-uniform: a longer row is another kernel's
  int32_t Q = 2;
  while (Q < L) Q <<= 1;
  const bool idle = wv * PW >= Q;  // wavefront-uniform
  int32_t x[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int32_t i = i0 + e * kWave;
    x[e] = i < L ? adj[beg + i] : kPad;
  }
  for (int k = 2; k <= Q; k <<= 1) {
#pragma unroll
    for (int j = P / 2; j > 0; j >>= 1) {
      if (j >= k) continue;  // block-uniform: the strides of stage k are k / 2 .. 1
      if (j >= PW) {
#pragma unroll
        for (int e = 0; e < E; ++e) s[i0 + e * kWave] = x[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int32_t i = i0 + e * kWave;
          const int32_t y = s[i ^ j];
          const bool up = (i & k) == 0;
          const bool lo = (i & j) == 0;
          x[e] = (lo == up) ? min(x[e], y) : max(x[e], y);
        }
        __syncthreads();
      } else if (idle) {
        continue;
      } else if (j >= kWave) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int pe = e ^ (j / kWave);
          if (pe > e) {
            const bool up = ((wv * PW + e * kWave) & k) == 0;  // k > 64: the lane bits do not matter
            const int32_t a = x[e], b = x[pe];
            x[e] = up ? min(a, b) : max(a, b);
            x[pe] = up ? max(a, b) : min(a, b);
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int32_t y = __shfl_xor(x[e], j, kWave);
          const bool up = ((i0 + e * kWave) & k) == 0;
          const bool lo = (lane & j) == 0;
          x[e] = (lo == up) ? min(x[e], y) : max(x[e], y);
        }
      }
    }
  }
  if (!DEDUP) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int32_t i = i0 + e * kWave;
      if (i < L) adj[beg + i] = x[e];
    }
    return;
  }
  // in-order dedup: the id before x[0] of lane 0 is the previous wavefront's
  // last; the unique flags are formed twice (count, then write) rather than
  // kept in registers
  if (lane == kWave - 1) wlast[wv] = x[E - 1];
  __syncthreads();
  const int32_t before = wv > 0 ? wlast[wv > 0 ? wv - 1 : 0] : 0;
  auto unique = [&](int e) -> uint64_t {
    const int32_t i = i0 + e * kWave;
    int32_t prev = __shfl_up(x[e], 1, kWave);
    if (lane == 0) prev = e > 0 ? __builtin_amdgcn_readlane(x[e > 0 ? e - 1 : 0], kWave - 1) : before;
    return __ballot(i < L && (i == 0 || x[e] != prev));
  };
  int32_t cnt = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) cnt += (int32_t)__popcll(unique(e));
  if (lane == 0) wsum[wv] = cnt;
  __syncthreads();
  int32_t base = 0;
  for (int q = 0; q < wv; ++q) base += wsum[q];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t um = unique(e);
    if ((um >> lane) & 1) adj[beg + base + mask_below(um)] = x[e];
    base += (int32_t)__popcll(um);
  }
  if (wv == W - 1 && lane == 0) deg[v] = base;
}

hipError_t launch_sort_rows(int cls, const int32_t* rows, int32_t nrows, const int64_t* off,
                            const int32_t* len, int32_t* adj, int32_t* deg, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  switch (cls) {
    case kRow8: k_sort_small<8><<<grid_for((int64_t)nrows * 8, 256, 1u << 30), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRow16: k_sort_small<16><<<grid_for((int64_t)nrows * 16, 256, 1u << 30), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRow32: k_sort_small<32><<<grid_for((int64_t)nrows * 32, 256, 1u << 30), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRow64: k_sort_small<64><<<grid_for((int64_t)nrows * 64, 256, 1u << 30), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRow128: k_sort_wave<2><<<grid_for((int64_t)nrows * kWave, 256, 1u << 16), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRow256: k_sort_wave<4><<<grid_for((int64_t)nrows * kWave, 256, 1u << 16), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRow512: k_sort_wave<8><<<grid_for((int64_t)nrows * kWave, 256, 1u << 16), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRow1024: k_sort_wave<16><<<grid_for((int64_t)nrows * kWave, 256, 1u << 16), 256, 0, s>>>(rows, nrows, off, len, adj, deg); break;
    case kRowLds4k: k_sort_block<16, 4, true><<<nrows, 256, 0, s>>>(rows, nullptr, nullptr, off, len, adj, deg); break;
    case kRowLds8k: k_sort_block<16, 8, true><<<nrows, 512, 0, s>>>(rows, nullptr, nullptr, off, len, adj, deg); break;
    case kRowLds32k:  // up to 16,384 ids in registers (32 per lane would spill), longer rows by the LDS network
      k_sort_block<16, 16, true><<<nrows, 1024, 0, s>>>(rows, nullptr, nullptr, off, len, adj, deg);
      k_sort_lds<kLargeChunk, 1024, true><<<nrows, 1024, 0, s>>>(rows, nullptr, nullptr, off, len, adj, deg,
                                                                 kWave * 16 * 16);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sort_chunks(const int64_t* chunk_beg, const int32_t* chunk_len, int32_t nchunks,
                              int32_t* buf, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  k_sort_lds<kLargeChunk, 1024, false><<<nchunks, 1024, 0, s>>>(nullptr, chunk_beg, chunk_len, nullptr, nullptr, buf,
                                                                 nullptr, 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Merge pass for large rows (merge path partition, A first on ties).
constexpr int kMergeItems = 8;
static_assert(kMergeTile == 256 * kMergeItems, "tile");

__global__ __launch_bounds__(256) void k_merge(const int64_t* __restrict__ a_beg, const int32_t* __restrict__ la_,
                                               const int32_t* __restrict__ lb_, const int64_t* __restrict__ out_beg,
                                               const int64_t* __restrict__ tile_off, int32_t njobs,
                                               const int32_t* __restrict__ in, int32_t* __restrict__ out) {
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = njobs - 1;  // job = last k with tile_off[k] <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_off[mid] <= tile) lo = mid; else hi = mid - 1;
  }
  const int job = lo;
  const int32_t la = la_[job], lb = lb_[job];
  const int32_t* A = in + a_beg[job];
  const int32_t* B = A + la;
  int32_t* O = out + out_beg[job];
  const int64_t k0l = (tile - tile_off[job]) * (int64_t)kMergeTile + (int64_t)threadIdx.x * kMergeItems;
  if (k0l >= (int64_t)la + lb) return;
  const int32_t k0 = (int32_t)k0l;
  int32_t b0 = max(0, k0 - lb), e0 = min(k0, la);
  while (b0 < e0) {
    const int32_t mid = (b0 + e0) >> 1;
    if (A[mid] <= B[k0 - 1 - mid]) b0 = mid + 1; else e0 = mid;
  }
  int32_t i = b0, j = k0 - b0;
#pragma unroll
  for (int t = 0; t < kMergeItems; ++t) {
    if (k0 + t >= la + lb) break;
    const bool takeA = j >= lb || (i < la && A[i] <= B[j]);
    O[k0 + t] = takeA ? A[i] : B[j];
    if (takeA) ++i; else ++j;
  }
}

hipError_t launch_merge_pass(const int64_t* a_beg, const int32_t* la, const int32_t* lb,
                             const int64_t* out_beg, const int64_t* tile_off, int32_t njobs,
                             int64_t ntiles, const int32_t* buf_in, int32_t* buf_out, hipStream_t s) {
  if (njobs == 0 || ntiles == 0) return hipSuccess;
  k_merge<<<(unsigned)ntiles, 256, 0, s>>>(a_beg, la, lb, out_beg, tile_off, njobs, buf_in, buf_out);
  return hipGetLastError();
}

constexpr int kDedupNT = 1024;
constexpr int kDedupPer = 4;  // consecutive entries per thread per step

__global__ __launch_bounds__(kDedupNT) void k_dedup_rows(const int32_t* __restrict__ rows,
                                                         const int64_t* __restrict__ seg_beg,
                                                         const int32_t* __restrict__ len,
                                                         const int32_t* __restrict__ sorted,
                                                         const int64_t* __restrict__ off,
                                                         int32_t* __restrict__ adj, int32_t* __restrict__ deg) {
  __shared__ int32_t lds_scan[kDedupNT / kWave + 1];
  const int32_t v = rows[blockIdx.x];
  const int32_t L = len[v];
  const int32_t* S = sorted + seg_beg[blockIdx.x];
  int32_t* D = adj + off[v];
  int32_t carry = 0;
  for (int base = 0; base < L; base += kDedupNT * kDedupPer) {
    const int i0 = base + threadIdx.x * kDedupPer;
    int32_t x[kDedupPer];
    bool u[kDedupPer];
    int32_t c = 0;
    int32_t prev = i0 > 0 && i0 - 1 < L ? S[i0 - 1] : kPad;
#pragma unroll
    for (int q = 0; q < kDedupPer; ++q) {
      const int i = i0 + q;
      x[q] = i < L ? S[i] : kPad;
      u[q] = i < L && (i == 0 || x[q] != prev);
      prev = x[q];
      c += u[q];
    }
    __syncthreads();  // every read of this step precedes the writes (S may alias D)
    int32_t tot;
    int32_t at = carry + block_excl_scan<int32_t, kDedupNT>(c, lds_scan, &tot);
#pragma unroll
    for (int q = 0; q < kDedupPer; ++q)
      if (u[q]) D[at++] = x[q];
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) deg[v] = carry;
}

hipError_t launch_dedup_rows(const int32_t* rows, const int64_t* seg_beg, int32_t nrows,
                             const int32_t* len, const int32_t* sorted, const int64_t* off,
                             int32_t* adj, int32_t* deg, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  k_dedup_rows<<<nrows, kDedupNT, 0, s>>>(rows, seg_beg, len, sorted, off, adj, deg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4: orientation in one pass over every row plus a copy. The pass counts
// d+(v) and partitions row v into the same span of `part`: N+(v) (ascending)
// from the front, N-(v) from the back in reverse order. After d+ and d- are
// scanned, the copy streams both parts to dcol[doff[v]..] and
// dincol[dinoff[v]..], each ascending. Rows of raw length <= kOrientShort:
// a group of kOrientG lanes per row, grid-stride; medium rows: a wavefront
// each; long rows: a block each (both listed contiguously by the row
// classes).
// Degree classes for the rank test: class(d) = 0 below 64, 1 below 512, 2
// below 4096, else 3, two bits per node (16 nodes per word, 4 MB for 2^24
// nodes, small enough to stay in L2). A class order agrees with the degree
// order, so w ranks above v whenever class(w) > class(v), and below it
// whenever class(w) < class(v); only nodes of one class need d(w) itself.
// At R-MAT 24 about 3 in 4 edges join nodes of different classes, which
// saves that many random gathers of d(w).
__device__ __forceinline__ uint32_t deg_class(int32_t d) {
  return (uint32_t)(d >= 64) + (uint32_t)(d >= 512) + (uint32_t)(d >= 4096);
}

// True when w ranks above v (rank = (key, id), key = d by default); kv, cv =
// key(v), class(key(v)). The classes agree with any key order, so the same
// test serves the degree order and a caller's order (e.g. degeneracy).
__device__ __forceinline__ bool ranks_above(int32_t kv, uint32_t cv, int32_t v, int32_t w,
                                            const int32_t* __restrict__ key, const uint32_t* __restrict__ cls) {
  const uint32_t cw = (cls[w >> 4] >> (2 * (w & 15))) & 3u;
  if (cw != cv) return cw > cv;
  return rank_below(kv, v, key[w], w);
}

__global__ __launch_bounds__(256) void k_deg_class(int32_t n, const int32_t* __restrict__ key,
                                                   uint32_t* __restrict__ cls) {
  const int64_t words = ((int64_t)n + 15) / 16;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += (int64_t)gridDim.x * blockDim.x) {
    uint32_t word = 0;
    for (int j = 0; j < 16; ++j) {
      const int64_t v = k * 16 + j;
      if (v < n) word |= deg_class(key[v]) << (2 * j);
    }
    cls[k] = word;
  }
}

constexpr int kOrientG = 8;
constexpr int32_t kOrientShort = 64;
constexpr int kOrientShortUnroll = 4;  // steps of G entries issued together (short rows)
constexpr int kOrientMedUnroll = 4;    // chunks of 64 entries issued together (medium rows)

template <typename T>
__device__ __forceinline__ T block_max(T x, T* lds) {
  constexpr int NW = 256 / kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
  if (lane_id() == 0) lds[threadIdx.x / kWave] = x;
  __syncthreads();
  T r = lds[0];
  for (int i = 1; i < NW; ++i) r = max(r, lds[i]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_orient_short(int32_t n, const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ len,
                                                      const int32_t* __restrict__ deg,
                                                      const int32_t* __restrict__ key,
                                                      const uint32_t* __restrict__ cls,
                                                      const int32_t* __restrict__ adj,
                                                      int32_t* __restrict__ dplus, int32_t* __restrict__ part,
                                                      int32_t* __restrict__ stats) {
  constexpr int G = kOrientG;
  __shared__ int32_t red[256 / kWave];
  const int64_t ngroups = (int64_t)gridDim.x * (256 / G);
  const int g = threadIdx.x % G;
  const int shift = lane_id() & ~(G - 1);
  int32_t mx_d = 0, mx_p = 0;
  for (int64_t v = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G; v < n; v += ngroups) {
    if (len[v] > kOrientShort) continue;
    const int32_t dv = deg[v], kv = key[v];
    const uint32_t cv = deg_class(kv);
    const int64_t rb = off[v];
    const int32_t* row = adj + rb;
    int32_t* prow = part + rb;
    int32_t c = 0;
    for (int32_t b = 0; b < dv; b += G * kOrientShortUnroll) {
      int32_t w[kOrientShortUnroll];
      bool f[kOrientShortUnroll];
#pragma unroll
      for (int q = 0; q < kOrientShortUnroll; ++q) {
        const int32_t i = b + q * G + g;
        w[q] = i < dv ? row[i] : 0;
      }
#pragma unroll
      for (int q = 0; q < kOrientShortUnroll; ++q) {
        const int32_t i = b + q * G + g;
        f[q] = i < dv && ranks_above(kv, cv, (int32_t)v, w[q], key, cls);
      }
#pragma unroll
      for (int q = 0; q < kOrientShortUnroll; ++q) {
        const int32_t i = b + q * G + g;
        const uint32_t mask = (uint32_t)(__ballot(f[q]) >> shift) & ((1u << G) - 1);
        const int32_t below = __popc(mask & ((1u << g) - 1));
        if (f[q]) prow[c + below] = w[q];
        else if (i < dv) prow[dv - 1 - (i - (c + below))] = w[q];
        c += __popc(mask);
      }
    }
    if (g == 0) dplus[v] = c;
    mx_d = max(mx_d, dv);
    mx_p = max(mx_p, c);
  }
  mx_d = block_max(mx_d, red);
  mx_p = block_max(mx_p, red);
  if (threadIdx.x == 0) {
    atomicMax(&stats[0], mx_d);
    atomicMax(&stats[1], mx_p);
  }
}

constexpr int kOrientLongNT = 1024;
constexpr int kOrientLongPer = 4;  // consecutive entries per thread per step

__global__ __launch_bounds__(kOrientLongNT) void k_orient_long(const int32_t* __restrict__ rows,
                                                               const int64_t* __restrict__ off,
                                                               const int32_t* __restrict__ deg,
                                                               const int32_t* __restrict__ key,
                                                               const uint32_t* __restrict__ cls,
                                                               const int32_t* __restrict__ adj,
                                                               int32_t* __restrict__ dplus,
                                                               int32_t* __restrict__ part,
                                                               int32_t* __restrict__ stats) {
  __shared__ int32_t lds[kOrientLongNT / kWave + 1];
  const int32_t v = rows[blockIdx.x];
  const int32_t dv = deg[v], kv = key[v];
  const uint32_t cv = deg_class(kv);
  const int64_t rb = off[v];
  const int32_t* row = adj + rb;
  int32_t* prow = part + rb;
  int32_t c = 0;
  for (int32_t b = 0; b < dv; b += kOrientLongNT * kOrientLongPer) {
    const int32_t i0 = b + threadIdx.x * kOrientLongPer;
    int32_t w[kOrientLongPer];
    bool f[kOrientLongPer];
    int32_t k = 0;
#pragma unroll
    for (int q = 0; q < kOrientLongPer; ++q) w[q] = i0 + q < dv ? row[i0 + q] : 0;
#pragma unroll
    for (int q = 0; q < kOrientLongPer; ++q) {
      f[q] = i0 + q < dv && ranks_above(kv, cv, v, w[q], key, cls);
      k += f[q];
    }
    int32_t tot;
    int32_t o = c + block_excl_scan<int32_t, kOrientLongNT>(k, lds, &tot);  // out-entries before i0
#pragma unroll
    for (int q = 0; q < kOrientLongPer; ++q) {
      const int32_t i = i0 + q;
      if (i >= dv) break;
      if (f[q]) prow[o++] = w[q];
      else prow[dv - 1 - (i - o)] = w[q];
    }
    c += tot;
  }
  if (threadIdx.x == 0) {
    dplus[v] = c;
    atomicMax(&stats[0], dv);
    atomicMax(&stats[1], c);
  }
}

// Rows of medium length: one wavefront per row (grid-stride), ballot-ordered
// compaction, no block barriers.
__global__ __launch_bounds__(256) void k_orient_medium(const int32_t* __restrict__ rows, int32_t nrows,
                                                       const int64_t* __restrict__ off,
                                                       const int32_t* __restrict__ deg,
                                                       const int32_t* __restrict__ key,
                                                       const uint32_t* __restrict__ cls,
                                                       const int32_t* __restrict__ adj,
                                                       int32_t* __restrict__ dplus, int32_t* __restrict__ part,
                                                       int32_t* __restrict__ stats) {
  __shared__ int32_t red[256 / kWave];
  const int64_t nwaves = (int64_t)gridDim.x * (256 / kWave);
  const int l = lane_id();
  int32_t mx_d = 0, mx_p = 0;
  for (int64_t r = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave; r < nrows; r += nwaves) {
    const int32_t v = rows[r];
    const int32_t dv = deg[v], kv = key[v];
    const uint32_t cv = deg_class(kv);
    const int64_t rb = off[v];
    const int32_t* row = adj + rb;
    int32_t* prow = part + rb;
    int32_t c = 0;
    // kOrientMedUnroll chunks of 64 entries per step: their row loads, then
    // their degree gathers, are issued together
    for (int32_t b = 0; b < dv; b += kWave * kOrientMedUnroll) {
      int32_t w[kOrientMedUnroll];
      bool f[kOrientMedUnroll];
#pragma unroll
      for (int q = 0; q < kOrientMedUnroll; ++q) {
        const int32_t i = b + q * kWave + l;
        w[q] = i < dv ? row[i] : 0;
      }
#pragma unroll
      for (int q = 0; q < kOrientMedUnroll; ++q) {
        const int32_t i = b + q * kWave + l;
        f[q] = i < dv && ranks_above(kv, cv, v, w[q], key, cls);
      }
#pragma unroll
      for (int q = 0; q < kOrientMedUnroll; ++q) {
        const int32_t i = b + q * kWave + l;
        const uint64_t m = __ballot(f[q]);
        const int32_t below = mask_below(m);
        if (f[q]) prow[c + below] = w[q];
        else if (i < dv) prow[dv - 1 - (i - (c + below))] = w[q];
        c += (int32_t)__popcll(m);
      }
    }
    if (l == 0) dplus[v] = c;
    mx_d = max(mx_d, dv);
    mx_p = max(mx_p, c);
  }
  mx_d = block_max(mx_d, red);
  mx_p = block_max(mx_p, red);
  if (threadIdx.x == 0) {
    atomicMax(&stats[0], mx_d);
    atomicMax(&stats[1], mx_p);
  }
}

// Copy of the partitioned rows: N+(v) = part[off[v] .. off[v] + d+(v)) to
// dcol[doff[v] ..]; N-(v) = part[off[v] + d(v) - 1 - k], k < d-(v), to
// dincol[dinoff[v] + k] (ascending again). G lanes per row (G = 8, 64 or
// 256), rows short (all rows of raw length <= kOrientShort, grid-stride),
// or listed.
template <int G>
__device__ __forceinline__ void orient_copy_row(int32_t v, int g, const int64_t* __restrict__ off,
                                                const int32_t* __restrict__ deg,
                                                const int32_t* __restrict__ dplus,
                                                const int32_t* __restrict__ part, const int64_t* __restrict__ doff,
                                                int32_t* __restrict__ dcol, const int64_t* __restrict__ dinoff,
                                                int32_t* __restrict__ dincol) {
  constexpr int U = 4;  // loads of each list issued together per step
  const int32_t dv = deg[v], dp = dplus[v];
  const int32_t di = dincol ? dv - dp : 0;
  const int32_t* prow = part + off[v];
  const int32_t* pend = prow + dv - 1;
  int32_t* out = dcol + doff[v];
  int32_t* in = dincol ? dincol + dinoff[v] : nullptr;
  const int32_t dm = max(dp, di);
  for (int32_t k0 = g; k0 < dm; k0 += G * U) {
    int32_t a[U], b[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int32_t k = k0 + q * G;
      a[q] = k < dp ? prow[k] : 0;
      b[q] = k < di ? pend[-k] : 0;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int32_t k = k0 + q * G;
      if (k < dp) out[k] = a[q];
      if (k < di) in[k] = b[q];
    }
  }
}

__global__ __launch_bounds__(256) void k_orient_copy_short(int32_t n, const int64_t* __restrict__ off,
                                                           const int32_t* __restrict__ len,
                                                           const int32_t* __restrict__ deg,
                                                           const int32_t* __restrict__ dplus,
                                                           const int32_t* __restrict__ part,
                                                           const int64_t* __restrict__ doff,
                                                           int32_t* __restrict__ dcol,
                                                           const int64_t* __restrict__ dinoff,
                                                           int32_t* __restrict__ dincol) {
  constexpr int G = kOrientG;
  const int64_t ngroups = (int64_t)gridDim.x * (256 / G);
  for (int64_t v = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G; v < n; v += ngroups) {
    if (len[v] > kOrientShort) continue;
    orient_copy_row<G>((int32_t)v, threadIdx.x % G, off, deg, dplus, part, doff, dcol, dinoff, dincol);
  }
}

template <int G>
__global__ __launch_bounds__(256) void k_orient_copy_listed(const int32_t* __restrict__ rows, int32_t nrows,
                                                            const int64_t* __restrict__ off,
                                                            const int32_t* __restrict__ deg,
                                                            const int32_t* __restrict__ dplus,
                                                            const int32_t* __restrict__ part,
                                                            const int64_t* __restrict__ doff,
                                                            int32_t* __restrict__ dcol,
                                                            const int64_t* __restrict__ dinoff,
                                                            int32_t* __restrict__ dincol) {
  const int64_t ngroups = (int64_t)gridDim.x * (256 / G);
  for (int64_t r = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G; r < nrows; r += ngroups)
    orient_copy_row<G>(rows[r], threadIdx.x % G, off, deg, dplus, part, doff, dcol, dinoff, dincol);
}

hipError_t launch_orient(int32_t n, const int64_t* off, const int32_t* len, const int32_t* deg, const int32_t* key,
                         const int32_t* adj, const int32_t* medium_rows, int32_t nmedium, const int32_t* long_rows,
                         int32_t nlong, uint32_t* cls, int32_t* dplus, int32_t* part, int32_t* stats, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (!key) key = deg;
  k_deg_class<<<grid_for(((int64_t)n + 15) / 16, 256, 4096), 256, 0, s>>>(n, key, cls);
  k_orient_short<<<grid_for((int64_t)n * kOrientG, 256, 1u << 16), 256, 0, s>>>(n, off, len, deg, key, cls, adj,
                                                                             dplus, part, stats);
  if (nmedium > 0)
    k_orient_medium<<<grid_for((int64_t)nmedium * kWave, 256, 1u << 14), 256, 0, s>>>(medium_rows, nmedium, off, deg,
                                                                                   key, cls, adj, dplus, part, stats);
  if (nlong > 0)
    k_orient_long<<<nlong, kOrientLongNT, 0, s>>>(long_rows, off, deg, key, cls, adj, dplus, part, stats);
  return hipGetLastError();
}

hipError_t launch_orient_copy(int32_t n, const int64_t* off, const int32_t* len, const int32_t* deg,
                              const int32_t* dplus, const int32_t* part, const int32_t* medium_rows, int32_t nmedium,
                              const int32_t* long_rows, int32_t nlong, const int64_t* doff, int32_t* dcol,
                              const int64_t* dinoff, int32_t* dincol, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_orient_copy_short<<<grid_for((int64_t)n * kOrientG, 256, 1u << 16), 256, 0, s>>>(n, off, len, deg, dplus, part,
                                                                                  doff, dcol, dinoff, dincol);
  if (nmedium > 0)
    k_orient_copy_listed<kWave><<<grid_for((int64_t)nmedium * kWave, 256, 1u << 14), 256, 0, s>>>(
        medium_rows, nmedium, off, deg, dplus, part, doff, dcol, dinoff, dincol);
  if (nlong > 0)
    k_orient_copy_listed<256><<<grid_for((int64_t)nlong * 256, 256, 1u << 14), 256, 0, s>>>(
        long_rows, nlong, off, deg, dplus, part, doff, dcol, dinoff, dincol);
  return hipGetLastError();
}

// d-(v) = d(v) - d+(v)
// d-(v) = d(v) - d+(v); *deg2 (zeroed) += the number of nodes with d >= 2.
__global__ __launch_bounds__(256) void k_indeg(int32_t n, const int32_t* __restrict__ deg,
                                               const int32_t* __restrict__ dplus, int32_t* __restrict__ din,
                                               int32_t* __restrict__ deg2) {
  __shared__ int32_t red[256 / kWave];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int32_t c = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t d = deg[v];
    din[v] = d - dplus[v];
    c += d >= 2;
  }
  const int32_t t = block_sum<int32_t, 256>(c, red);
  if (threadIdx.x == 0 && t) atomicAdd(deg2, t);
}

hipError_t launch_indeg(int32_t n, const int32_t* deg, const int32_t* dplus, int32_t* din, int32_t* deg2,
                        hipStream_t s) {
  if (n == 0) return hipSuccess;
  // few blocks: each ends with one atomic on the shared counter
  k_indeg<<<grid_for(n, 256 * 16, 2048), 256, 0, s>>>(n, deg, dplus, din, deg2);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Graphs handed over as a CSR (rows d_col[rowptr[v] .. rowptr[v+1])).
// k_csr_bounds: rowptr[0] == 0, non-decreasing, rowptr[n] == nnz (else bit
// 4 of err); len = deg = row lengths. Rows are read only after this passed.
__global__ __launch_bounds__(256) void k_csr_bounds(int32_t n, int64_t nnz, const int64_t* __restrict__ rowptr,
                                                    int32_t* __restrict__ len, int32_t* __restrict__ deg,
                                                    int32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t b = rowptr[v], e = rowptr[v + 1];
    if (b > e || b < 0 || e > nnz || (v == 0 && b != 0) || (v == n - 1 && e != nnz)) bad = true;
    const int32_t l = bad ? 0 : (int32_t)(e - b);
    if (len) len[v] = l;
    if (deg) deg[v] = l;
  }
  if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0 && (rowptr[0] != 0 || nnz != 0)) bad = true;
  if (__ballot(bad) && lane_id() == 0) atomicOr(err, 4);
}

// One wavefront per row: ids in [0, n) (else bit 1), strictly ascending and
// without the row's own id (else bit 2).
__global__ __launch_bounds__(256) void k_csr_rows(int32_t n, const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col, int32_t* __restrict__ err) {
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
  bool range = false, order = false;
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < n; v += nw) {
    const int64_t b = rowptr[v], e = rowptr[v + 1];
    for (int64_t i = b + lane; i < e; i += kWave) {
      const int32_t x = col[i];
      if ((uint32_t)x >= (uint32_t)n) range = true;
      if (x == (int32_t)v || (i > b && col[i - 1] >= x)) order = true;
    }
  }
  const uint64_t r = __ballot(range), o = __ballot(order);
  if (lane == 0 && (r | o)) atomicOr(err, (r ? 1 : 0) | (o ? 2 : 0));
}

// src[i] = v for every entry i of row v: the CSR as a list of (v, w) pairs.
__global__ __launch_bounds__(256) void k_csr_expand(int32_t n, const int64_t* __restrict__ rowptr,
                                                    int32_t* __restrict__ src) {
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < n; v += nw) {
    const int64_t b = rowptr[v], e = rowptr[v + 1];
    for (int64_t i = b + lane; i < e; i += kWave) src[i] = (int32_t)v;
  }
}

hipError_t launch_csr_bounds(int32_t n, int64_t nnz, const int64_t* rowptr, int32_t* len, int32_t* deg, int32_t* err,
                             hipStream_t s) {
  k_csr_bounds<<<grid_for(n > 0 ? n : 1, 256, 1u << 16), 256, 0, s>>>(n, nnz, rowptr, len, deg, err);
  return hipGetLastError();
}

hipError_t launch_csr_rows(int32_t n, const int64_t* rowptr, const int32_t* col, int32_t* err, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_csr_rows<<<grid_for(n, 4, 1u << 16), 256, 0, s>>>(n, rowptr, col, err);
  return hipGetLastError();
}

hipError_t launch_csr_expand(int32_t n, const int64_t* rowptr, int32_t* src, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_csr_expand<<<grid_for(n, 4, 1u << 16), 256, 0, s>>>(n, rowptr, src);
  return hipGetLastError();
}

// Work items of the in-list pass: the nodes w of one bin (listed
// contiguously) each get ceil(d-(w) / chunk) items.
__global__ __launch_bounds__(256) void k_in_chunks(const int32_t* __restrict__ list, int64_t nlist,
                                                   const int32_t* __restrict__ din, const int32_t* __restrict__ cap_of,
                                                   const int64_t* __restrict__ bin_off, int32_t* __restrict__ nch) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nlist; i += stride) {
    int b = 0;
    while (b < kNumBins - 1 && i >= bin_off[b + 1]) ++b;
    const int32_t c = max(1, cap_of[b]);
    nch[i] = (din[list[i]] + c - 1) / c;
  }
}

hipError_t launch_in_chunks(const int32_t* list, int64_t nlist, const int32_t* din, const int32_t* cap_of,
                            const int64_t* bin_off, int32_t* nch, hipStream_t s) {
  if (nlist == 0) return hipSuccess;
  k_in_chunks<<<grid_for(nlist, 256, 1u << 14), 256, 0, s>>>(list, nlist, din, cap_of, bin_off, nch);
  return hipGetLastError();
}

// Chunk -> owner map of the in-list items, so that a work item finds its
// owner with one load instead of a search over the chunk prefix.
__global__ __launch_bounds__(256) void k_in_owners(int64_t nlist, const int64_t* __restrict__ coff,
                                                   int32_t* __restrict__ owner) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nlist; i += stride)
    for (int64_t c = coff[i]; c < coff[i + 1]; ++c) owner[c] = (int32_t)i;
}

hipError_t launch_in_owners(int64_t nlist, const int64_t* coff, int32_t* owner, hipStream_t s) {
  if (nlist == 0) return hipSuccess;
  k_in_owners<<<grid_for(nlist, 256, 1u << 14), 256, 0, s>>>(nlist, coff, owner);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sum over DAG edges u->w of d+(u) + d+(w): the list elements a merge-based
// intersection reads (the algorithmic-bytes measure of the hot loop).
__global__ __launch_bounds__(256) void k_list_elems(int32_t n, const int64_t* __restrict__ doff,
                                                    const int32_t* __restrict__ dcol,
                                                    unsigned long long* __restrict__ out) {
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int l = lane_id();
  unsigned long long acc = 0;
  for (int64_t u = w0; u < n; u += nwaves) {
    const int64_t b = doff[u], e = doff[u + 1];
    const unsigned long long du = (unsigned long long)(e - b);
    for (int64_t p = b + l; p < e; p += kWave) {
      const int32_t w = dcol[p];
      acc += du + (unsigned long long)(doff[w + 1] - doff[w]);
    }
  }
  acc = group_sum<unsigned long long, kWave>(acc);
  if (l == 0 && acc) atomicAdd(out, acc);
}

hipError_t launch_list_elems(int32_t n, const int64_t* doff, const int32_t* dcol, unsigned long long* out,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_list_elems<<<grid_for((int64_t)n * kWave, 256, 1u << 14), 256, 0, s>>>(n, doff, dcol, out);
  return hipGetLastError();
}

// Per-bin algorithmic sizes: every DAG edge u->w with d+(u) >= 2 is charged
// to the bin whose kernel counts it: w's bin (by d+(w)) when the min-side
// rule hands it to w's in-list (d+(u) < d+(w) <= w_max), else u's bin.
// elems[b] += d+(u) + d+(w), edges[b] += 1. Wave per node, grid-stride.
__device__ __forceinline__ int bin_of(int32_t d, const int32_t* lim) {
  int b = kNumBins - 1;
#pragma unroll
  for (int q = kNumBins - 2; q >= 0; --q)
    if (d <= lim[q]) b = q;
  return b;
}

// Per bin b, over the DAG edges u->w that bin b's kernel counts (min-side
// ownership with w_max; w_max = 0 counts every edge from its tail):
//   elems[b]  sum of d+(u) + d+(w) (what a merge of both lists reads)
//   edges[b]  number of such edges
//   kbytes[b] bytes the min-side kernel moves for the bin when nothing is
//             reused between its work items: per out-list item u, its row
//             bounds (16), N+(u) for the table (4 d+(u)), the row bounds of
//             every w (16 d+(u)) and the T credits (8 (d+(u) + 1)); per
//             streamed list its ids (4 per id); per in-list chunk of w (din
//             in-neighbours, chunks of cap[b]), its bounds (32), N+(w) for
//             the table and the credits (12 d+(w) + 8); per in-neighbour its
//             entry and row bounds (20) and, if its list is streamed, its
//             credit (8).
__global__ __launch_bounds__(256) void k_bin_elems(int32_t n, const int64_t* __restrict__ doff,
                                                   const int32_t* __restrict__ dcol,
                                                   const int32_t* __restrict__ din,
                                                   const int32_t* __restrict__ limit,
                                                   const int32_t* __restrict__ cap, int32_t w_max,
                                                   unsigned long long* __restrict__ elems,
                                                   unsigned long long* __restrict__ edges,
                                                   unsigned long long* __restrict__ kbytes) {
  int32_t lim[kNumBins - 1];
#pragma unroll
  for (int q = 0; q < kNumBins - 1; ++q) lim[q] = limit[q];
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int l = lane_id();
  unsigned long long acc[kNumBins] = {}, eacc[kNumBins] = {}, kacc[kNumBins] = {};
  for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; u < n; u += nwaves) {
    const int64_t beg = doff[u], end = doff[u + 1];
    const int32_t du = (int32_t)(end - beg);
    const int bu = bin_of(du, lim);
    if (l == 0) {
      unsigned long long kb = 0;
      if (du >= 2) kb += 16ull + 28ull * (unsigned long long)du + 8ull;
      const int32_t di = din ? din[u] : 0;
      if (w_max > 0 && du >= 3 && du <= w_max && di >= 1) {
        const int32_t c = max(1, cap[bu]);
        const unsigned long long chunks = (unsigned long long)((di + c - 1) / c);
        kb += chunks * (40ull + 12ull * (unsigned long long)du) + 20ull * (unsigned long long)di;
      }
#pragma unroll
      for (int q = 0; q < kNumBins; ++q)
        if (q == bu) kacc[q] += kb;
    }
    if (du < 2) continue;
    for (int64_t p = beg + l; p < end; p += kWave) {
      const int32_t w = dcol[p];
      const int32_t dw = (int32_t)(doff[w + 1] - doff[w]);
      const bool in_side = du < dw && dw <= w_max;
      const int b = in_side ? bin_of(dw, lim) : bu;
      const unsigned long long kb = in_side ? 4ull * (unsigned long long)du + 8ull : 4ull * (unsigned long long)dw;
#pragma unroll
      for (int q = 0; q < kNumBins; ++q)
        if (q == b) { acc[q] += (unsigned long long)(du + dw); eacc[q] += 1; kacc[q] += kb; }
    }
  }
#pragma unroll
  for (int q = 0; q < kNumBins; ++q) {
    const unsigned long long a = group_sum<unsigned long long, kWave>(acc[q]);
    const unsigned long long e = group_sum<unsigned long long, kWave>(eacc[q]);
    const unsigned long long k = group_sum<unsigned long long, kWave>(kacc[q]);
    if (l == 0 && a) atomicAdd(&elems[q], a);
    if (l == 0 && e) atomicAdd(&edges[q], e);
    if (l == 0 && k) atomicAdd(&kbytes[q], k);
  }
}

hipError_t launch_bin_elems(int32_t n, const int64_t* doff, const int32_t* dcol, const int32_t* din,
                            const int32_t* limit, const int32_t* cap, int32_t w_max, unsigned long long* elems,
                            unsigned long long* edges, unsigned long long* kbytes, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_bin_elems<<<grid_for((int64_t)n * kWave, 256, 1u << 14), 256, 0, s>>>(n, doff, dcol, din, limit, cap, w_max,
                                                                         elems, edges, kbytes);
  return hipGetLastError();
}

// Streaming copy, 16 bytes per lane per iteration (the bandwidth probe).
__global__ __launch_bounds__(256) void k_probe_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                    int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

hipError_t launch_probe_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  k_probe_copy<<<grid_for(n16, 256 * 4, 8192), 256, 0, s>>>(static_cast<uint4*>(dst),
                                                            static_cast<const uint4*>(src), n16);
  return hipGetLastError();
}

// Packed batch -> disjoint union: the graph of edge e is found by binary
// search over edge_off (G + 1 entries). With src null only dst is mapped (the
// column array of a packed CSR, whose rows already sit at global positions).
__global__ __launch_bounds__(256) void k_batch_relabel(int32_t G, const int64_t* __restrict__ node_off,
                                                       const int64_t* __restrict__ edge_off,
                                                       const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ dst, int64_t m_raw,
                                                       int32_t* __restrict__ gsrc, int32_t* __restrict__ gdst,
                                                       int32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m_raw; e += stride) {
    int32_t lo = 0, hi = G - 1;  // last g with edge_off[g] <= e
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (edge_off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int64_t base = node_off[lo];
    const int64_t ng = node_off[lo + 1] - base;
    const int32_t u = src ? src[e] : 0, v = dst[e];
    if (u < 0 || v < 0 || u >= ng || v >= ng) {
      bad = true;
      if (src) gsrc[e] = (int32_t)base;  // keeps the union well formed; the build is refused anyway
      gdst[e] = (int32_t)base;
      continue;
    }
    if (src) gsrc[e] = (int32_t)(base + u);
    gdst[e] = (int32_t)(base + v);
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(err, 1);
}

hipError_t launch_batch_relabel(int32_t num_graphs, const int64_t* node_off, const int64_t* edge_off,
                                const int32_t* src, const int32_t* dst, int64_t m_raw, int32_t* gsrc,
                                int32_t* gdst, int32_t* err, hipStream_t s) {
  if (m_raw == 0) return hipSuccess;
  k_batch_relabel<<<grid_for(m_raw, 256 * 8, 1u << 16), 256, 0, s>>>(num_graphs, node_off, edge_off, src, dst,
                                                                     m_raw, gsrc, gdst, err);
  return hipGetLastError();
}

__global__ void k_gather_rows(const int32_t* __restrict__ rows, int32_t nr, const int64_t* __restrict__ off,
                              const int32_t* __restrict__ len, int64_t* __restrict__ out_off,
                              int32_t* __restrict__ out_len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr) { out_off[i] = off[rows[i]]; out_len[i] = len[rows[i]]; }
}

hipError_t launch_gather_rows(const int32_t* rows, int32_t nr, const int64_t* off, const int32_t* len,
                              int64_t* out_off, int32_t* out_len, hipStream_t s) {
  if (nr == 0) return hipSuccess;
  k_gather_rows<<<(nr + 255) / 256, 256, 0, s>>>(rows, nr, off, len, out_off, out_len);
  return hipGetLastError();
}

}  // namespace tricc

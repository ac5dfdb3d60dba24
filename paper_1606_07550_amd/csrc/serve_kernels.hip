// Induced-subgraph extraction for query batches (subgraph extraction is one
// of the graph manipulation methods in the paper's table of methods,
// Section 4; node ids keep their identity, Section 3.1).
//
// A batch holds Q queries; query q is the node set S_q = nodes[qoff[q] ..
// qoff[q+1]) of the resident graph (distinct ids), and its induced subgraph
// G[S_q] gets local ids = positions in S_q. Every undirected edge {v,w} of
// the resident graph with v, w in S_q and v < w (by id) is emitted once as
// the pair (pos(v), pos(w)).
//
// Membership is a per-query open-addressing table in global memory (key =
// node id, value = position; 2^k >= 2|S_q| slots). Rows of the resident CSR
// are scanned in chunks of kChunk neighbours, one wavefront per (item,
// chunk), so hub rows spread over many waves. Exact counts per chunk, a
// prefix sum, then an ordered fill give a deterministic pair list.
#include "device_common.h"
#include "kernels.h"

namespace tricc {

constexpr int32_t kServeChunk = 2048;

namespace {

// query of flat item i: last q with qoff[q] <= i
__device__ __forceinline__ int32_t find_query(const int64_t* qoff, int32_t Q, int64_t i) {
  int32_t lo = 0, hi = Q - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (qoff[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ uint32_t qhash(int32_t x) { return (uint32_t)x * 0x9E3779B1u; }

__device__ __forceinline__ int32_t table_lookup(const int2* tab, uint32_t mask, int32_t x) {
  uint32_t h = qhash(x) & mask;
  while (true) {
    const int2 e = tab[h];
    if (e.x == x) return e.y;
    if (e.x < 0) return -1;
    h = (h + 1) & mask;
  }
}

}  // namespace

// Clears every query table (key -1).
__global__ __launch_bounds__(256) void k_serve_clear(int2* __restrict__ tab, int64_t total) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) tab[i] = make_int2(-1, -1);
}

// Inserts every (node, position) and writes the number of row chunks and
// the query of each item; flags node ids outside [0, n) or repeated inside
// one query.
__global__ __launch_bounds__(256) void k_serve_insert(int32_t Q, const int64_t* __restrict__ qoff,
                                                      const int32_t* __restrict__ nodes,
                                                      const int64_t* __restrict__ toff, int2* __restrict__ tab,
                                                      int32_t n, const int32_t* __restrict__ deg,
                                                      int32_t* __restrict__ nchunks, int32_t* __restrict__ qidx,
                                                      int32_t* __restrict__ err) {
  const int64_t N = qoff[Q];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    const int32_t q = find_query(qoff, Q, i);
    qidx[i] = q;
    const int32_t v = nodes[i];
    if ((uint32_t)v >= (uint32_t)n) {
      atomicOr(err, 1);
      nchunks[i] = 0;
      continue;
    }
    int2* t = tab + toff[q];
    const uint32_t mask = (uint32_t)(toff[q + 1] - toff[q] - 1);
    uint32_t h = qhash(v) & mask;
    while (true) {
      const int prev = atomicCAS(&t[h].x, -1, v);
      if (prev == -1) { t[h].y = (int32_t)(i - qoff[q]); break; }
      if (prev == v) { atomicOr(err, 2); break; }
      h = (h + 1) & mask;
    }
    nchunks[i] = (deg[v] + kServeChunk - 1) / kServeChunk;
  }
}

// Item of every row chunk (the chunk prefix coff inverted), so that a
// chunk finds its item with one load instead of a search.
__global__ __launch_bounds__(256) void k_serve_items(int64_t N, const int64_t* __restrict__ coff,
                                                     int32_t* __restrict__ item) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    for (int64_t c = coff[i]; c < coff[i + 1]; ++c) item[c] = (int32_t)i;
}

// One wavefront per (item, chunk): pass 0 counts the emitted pairs of the
// chunk into cnt[c]; pass 1 writes them, in row order, at pos[c].
__global__ __launch_bounds__(256) void k_serve_pairs(int pass, int32_t Q, const int64_t* __restrict__ qoff,
                                                     const int32_t* __restrict__ nodes,
                                                     const int64_t* __restrict__ coff,  // chunk prefix per item
                                                     const int32_t* __restrict__ item,  // item of each chunk
                                                     const int32_t* __restrict__ qidx,  // query of each item
                                                     const int64_t* __restrict__ toff,
                                                     const int2* __restrict__ tab, const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ deg,
                                                     const int32_t* __restrict__ adj,
                                                     int32_t* __restrict__ cnt, const int64_t* __restrict__ pos,
                                                     int32_t* __restrict__ psrc, int32_t* __restrict__ pdst) {
  const int64_t N = qoff[Q];
  const int64_t C = coff[N];
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int l = lane_id();
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; c < C; c += nwaves) {
    const int64_t i = item[c];
    const int32_t q = qidx[i];
    const int32_t v = nodes[i];
    const int32_t pv = (int32_t)(i - qoff[q]);
    const int2* t = tab + toff[q];
    const uint32_t mask = (uint32_t)(toff[q + 1] - toff[q] - 1);
    const int32_t dv = deg[v];
    const int32_t b0 = (int32_t)(c - coff[i]) * kServeChunk;
    const int32_t b1 = min(dv, b0 + kServeChunk);
    const int32_t* row = adj + off[v];
    int32_t k = 0;
    int64_t base = pass == 1 ? pos[c] : 0;
    for (int32_t b = b0; b < b1; b += kWave) {
      int32_t pw = -1;
      if (b + l < b1) {
        const int32_t w = row[b + l];
        if (w > v) pw = table_lookup(t, mask, w);
      }
      const uint64_t m = __ballot(pw >= 0);
      if (pass == 1 && pw >= 0) {
        const int64_t at = base + k + mask_below(m);
        psrc[at] = pv;
        pdst[at] = pw;
      }
      k += (int32_t)__popcll(m);
    }
    if (pass == 0 && l == 0) cnt[c] = k;
  }
}

// pair offsets of each query: pairs of query q start at pos[coff[qoff[q]]]
__global__ void k_serve_query_pairs(int32_t Q, const int64_t* __restrict__ qoff, const int64_t* __restrict__ coff,
                                    const int64_t* __restrict__ pos, int64_t* __restrict__ qpairs) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q <= Q) qpairs[q] = pos[coff[qoff[q]]];
}

hipError_t launch_serve_clear(int2* tab, int64_t total, hipStream_t s) {
  if (total == 0) return hipSuccess;
  k_serve_clear<<<grid_for(total, 256, 1u << 14), 256, 0, s>>>(tab, total);
  return hipGetLastError();
}

hipError_t launch_serve_insert(int32_t Q, const int64_t* qoff, const int32_t* nodes, int64_t N, const int64_t* toff,
                               int2* tab, int32_t n, const int32_t* deg, int32_t* nchunks, int32_t* qidx, int32_t* err,
                               hipStream_t s) {
  if (N == 0) return hipSuccess;
  k_serve_insert<<<grid_for(N, 256, 1u << 14), 256, 0, s>>>(Q, qoff, nodes, toff, tab, n, deg, nchunks, qidx, err);
  return hipGetLastError();
}

hipError_t launch_serve_items(int64_t N, const int64_t* coff, int32_t* item, hipStream_t s) {
  if (N == 0) return hipSuccess;
  k_serve_items<<<grid_for(N, 256, 1u << 14), 256, 0, s>>>(N, coff, item);
  return hipGetLastError();
}

hipError_t launch_serve_pairs(int pass, int32_t Q, const int64_t* qoff, const int32_t* nodes, const int64_t* coff,
                              int64_t C, const int32_t* item, const int32_t* qidx, const int64_t* toff, const int2* tab,
                              const int64_t* off, const int32_t* deg, const int32_t* adj, int32_t* cnt,
                              const int64_t* pos, int32_t* psrc, int32_t* pdst, hipStream_t s) {
  if (C == 0) return hipSuccess;
  k_serve_pairs<<<grid_for(C * kWave, 256, 1u << 14), 256, 0, s>>>(pass, Q, qoff, nodes, coff, item, qidx, toff, tab,
                                                                   off, deg, adj, cnt, pos, psrc, pdst);
  return hipGetLastError();
}

hipError_t launch_serve_query_pairs(int32_t Q, const int64_t* qoff, const int64_t* coff, const int64_t* pos,
                                    int64_t* qpairs, hipStream_t s) {
  k_serve_query_pairs<<<(Q + 1 + 255) / 256, 256, 0, s>>>(Q, qoff, coff, pos, qpairs);
  return hipGetLastError();
}

}  // namespace tricc

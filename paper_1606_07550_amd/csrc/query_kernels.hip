// Edge-existence tests over the simple graph's sorted rows (IsEdge, among
// the graph methods of Section 4). Section 5.1 tests an edge by a search in
// a node's sorted neighbour vector, O(log deg_max) in its complexity table;
// here each lane takes one query and searches the shorter of the two rows,
// so the cost is O(log min(d(u), d(v))) dependent loads.
#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

// True when key is in row[0, len) (ascending, unique). Binary search that
// stops as soon as it meets the key.
__device__ __forceinline__ bool row_has(const int32_t* __restrict__ row, int32_t len, int32_t key) {
  int32_t lo = 0, hi = len;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    const int32_t x = row[mid];
    if (x == key) return true;
    if (x < key) lo = mid + 1;
    else hi = mid;
  }
  return false;
}

constexpr int kQueryNT = 256;

// rec[v] = (row start of v as uint32, d(v)): one 8-byte load gives both,
// so a query fetches its two records in one round trip.
__global__ __launch_bounds__(kQueryNT) void k_edge_records(int32_t n, const int64_t* __restrict__ off,
                                                           const int32_t* __restrict__ deg, int2* __restrict__ rec) {
  const int64_t stride = (int64_t)gridDim.x * kQueryNT;
  for (int64_t v = (int64_t)blockIdx.x * kQueryNT + threadIdx.x; v < n; v += stride)
    rec[v] = make_int2((int32_t)(uint32_t)off[v], deg[v]);
}

// One query per thread (grid-stride): out[i] = 1 if {u[i], v[i]} is an edge,
// 0 if not (u == v included), kEdgeQueryBadId if an id is outside [0, n).
__global__ __launch_bounds__(kQueryNT) void k_has_edges(int64_t q, const int32_t* __restrict__ qu,
                                                        const int32_t* __restrict__ qv, int32_t n,
                                                        const int2* __restrict__ rec,
                                                        const int32_t* __restrict__ adj,
                                                        uint8_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kQueryNT;
  for (int64_t i = (int64_t)blockIdx.x * kQueryNT + threadIdx.x; i < q; i += stride) {
    const int32_t u = qu[i], v = qv[i];
    uint8_t r = 0;
    if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n) {
      r = kEdgeQueryBadId;
    } else if (u != v) {
      const int2 ru = rec[u], rv = rec[v];
      const bool su = ru.y <= rv.y;  // search the shorter row
      const int2 ra = su ? ru : rv;
      r = row_has(adj + (uint32_t)ra.x, ra.y, su ? v : u) ? 1 : 0;
    }
    out[i] = r;
  }
}

}  // namespace

hipError_t launch_edge_records(int32_t n, const int64_t* off, const int32_t* deg, int32_t* rec, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = ((int64_t)n + kQueryNT - 1) / kQueryNT;
  if (blocks > 4096) blocks = 4096;
  k_edge_records<<<(unsigned)blocks, kQueryNT, 0, s>>>(n, off, deg, reinterpret_cast<int2*>(rec));
  return hipGetLastError();
}

hipError_t launch_has_edges(int64_t q, const int32_t* qu, const int32_t* qv, int32_t n, const int32_t* rec,
                            const int32_t* adj, uint8_t* out, hipStream_t s) {
  if (q <= 0) return hipSuccess;
  int64_t blocks = (q + kQueryNT - 1) / kQueryNT;
  if (blocks > (int64_t(1) << 20)) blocks = int64_t(1) << 20;
  k_has_edges<<<(unsigned)blocks, kQueryNT, 0, s>>>(q, qu, qv, n, reinterpret_cast<const int2*>(rec), adj, out);
  return hipGetLastError();
}

}  // namespace tricc

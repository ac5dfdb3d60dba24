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

// One query per thread (grid-stride): out[i] = 1 if {u[i], v[i]} is an edge,
// 0 if not (u == v included), kEdgeQueryBadId if an id is outside [0, n).
__global__ __launch_bounds__(kQueryNT) void k_has_edges(int64_t q, const int32_t* __restrict__ qu,
                                                        const int32_t* __restrict__ qv, int32_t n,
                                                        const int64_t* __restrict__ off,
                                                        const int32_t* __restrict__ deg,
                                                        const int32_t* __restrict__ adj,
                                                        uint8_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kQueryNT;
  for (int64_t i = (int64_t)blockIdx.x * kQueryNT + threadIdx.x; i < q; i += stride) {
    const int32_t u = qu[i], v = qv[i];
    uint8_t r = 0;
    if ((uint32_t)u >= (uint32_t)n || (uint32_t)v >= (uint32_t)n) {
      r = kEdgeQueryBadId;
    } else if (u != v) {
      const int32_t du = deg[u], dv = deg[v];
      const bool su = du <= dv;  // search the shorter row
      const int32_t a = su ? u : v;
      r = row_has(adj + off[a], su ? du : dv, su ? v : u) ? 1 : 0;
    }
    out[i] = r;
  }
}

}  // namespace

hipError_t launch_has_edges(int64_t q, const int32_t* qu, const int32_t* qv, int32_t n, const int64_t* off,
                            const int32_t* deg, const int32_t* adj, uint8_t* out, hipStream_t s) {
  if (q <= 0) return hipSuccess;
  int64_t blocks = (q + kQueryNT - 1) / kQueryNT;
  if (blocks > (int64_t(1) << 20)) blocks = int64_t(1) << 20;
  k_has_edges<<<(unsigned)blocks, kQueryNT, 0, s>>>(q, qu, qv, n, off, deg, adj, out);
  return hipGetLastError();
}

}  // namespace tricc

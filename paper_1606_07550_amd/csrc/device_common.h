// Device-side helpers shared by the gfx950 kernels of this library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tricc {

constexpr int kWave = 64;
constexpr int32_t kPad = 0x7fffffff;  // sort padding; node ids are < 2^31 - 1

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Blocks for `work` items at per_block items each, at least 1, at most cap
// (grid-stride kernels cover the rest).
inline unsigned grid_for(int64_t work, int per_block, unsigned cap = 1u << 20) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (int64_t)cap) g = cap;
  return (unsigned)g;
}

// Orders the LDS traffic of one wavefront: all lanes of a wave run in lockstep,
// so a fence plus a scheduling barrier is enough between a write by one lane
// and a read by another lane of the same wave.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of set bits of `mask` strictly below this lane.
__device__ __forceinline__ int mask_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (l >= o) x += y;
  }
  return x;
}

template <typename T, int W>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, W);
  return x;
}

// Exclusive scan over a block of NT threads (NT a multiple of 64, <= 1024).
// Returns the exclusive prefix; *total receives the block sum.
// `lds` must hold NT/64 + 1 elements. Contains __syncthreads().
template <typename T, int NT>
__device__ __forceinline__ T block_excl_scan(T x, T* lds, T* total) {
  constexpr int NW = NT / kWave;
  const int w = threadIdx.x / kWave, l = lane_id();
  T inc = wave_incl_scan(x);
  if (l == kWave - 1) lds[w] = inc;
  __syncthreads();
  if (w == 0) {
    T v = l < NW ? lds[l] : T(0);
    T s = wave_incl_scan(v);
    if (l < NW) lds[l] = s - v;
    if (l == NW - 1) lds[NW] = s;
  }
  __syncthreads();
  T r = lds[w] + inc - x;
  *total = lds[NW];
  __syncthreads();
  return r;
}

// Sum over a block of NT threads in a fixed order (deterministic).
template <typename T, int NT>
__device__ __forceinline__ T block_sum(T x, T* lds) {
  constexpr int NW = NT / kWave;
  const int w = threadIdx.x / kWave, l = lane_id();
  x = group_sum<T, kWave>(x);
  if (l == 0) lds[w] = x;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0)
    for (int i = 0; i < NW; ++i) r += lds[i];
  __syncthreads();
  return r;  // valid in thread 0
}

// Hash of a node id onto `bits` bits (1 <= bits <= 20): multiply the low 24
// bits by an odd 24-bit constant with the full-rate 24-bit multiplier and
// keep the top bits of the low product word, each of which depends on all 24
// input bits. Ids that differ only above bit 23 share a home bucket, which
// costs a probe step at most. Unsigned throughout: a signed product shifted
// right would sign-extend past the table.
__device__ __forceinline__ uint32_t hash_slot(int32_t x, int bits) {
  return (((uint32_t)x & 0xFFFFFFu) * 0x9E3779u) >> (32 - bits);
}

// Third dword of a raw (unformatted, stride 0) gfx9 buffer resource: 32-bit
// data, loads past num_records bytes return 0 without a memory access.
constexpr int32_t kRawBufferWord3 = 0x00020000;

// Degree-order rank test: (d(a), a) < (d(b), b).
__device__ __forceinline__ bool rank_below(int32_t da, int32_t a, int32_t db, int32_t b) {
  return da < db || (da == db && a < b);
}

}  // namespace tricc

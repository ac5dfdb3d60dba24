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
#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace tricc {

namespace {

template <int G>
__device__ __forceinline__ void group_sync() {
  if constexpr (G > kWave) __syncthreads();
  else wave_sync();
}

// The triangle total is accumulated apart from the per-node counts T: each
// triangle is found by exactly one node group (at its DAG edge u->w, as a
// common x), and that group adds the number it found to one of kTotSlots
// counters, chosen by block so that no single address takes every atomic.
__device__ __forceinline__ void credit_total(unsigned long long* tot, unsigned long long t) {
  if (t) atomicAdd(&tot[blockIdx.x & (kTotSlots - 1)], t);
}

// Open-addressing table of NB buckets of 4 int32 keys (-1 = empty), probed
// bucket by bucket: a lookup is normally one 16-byte LDS read.
template <int NB>
__device__ __forceinline__ int bucket_insert(int32_t* K, int32_t x) {
  uint32_t b = hash_slot(x, __builtin_ctz(NB));
  while (true) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (atomicCAS(&K[4 * b + j], -1, x) == -1) return (int)(4 * b + j);
    b = (b + 1) & (NB - 1);
  }
}

// Slot of x, or -1. `first` is the already-loaded bucket hash_slot(x).
template <int NB>
__device__ __forceinline__ int bucket_match(const int4* Kb, int32_t x, uint32_t b, int4 q) {
  while (true) {
    if (q.x == x) return (int)(4 * b);
    if (q.y == x) return (int)(4 * b + 1);
    if (q.z == x) return (int)(4 * b + 2);
    if (q.w == x) return (int)(4 * b + 3);
    if (q.w < 0) return -1;  // keys fill a bucket in order: an empty last slot ends the chain
    b = (b + 1) & (NB - 1);
    q = Kb[b];
  }
}

template <int SLOTS>
__device__ __forceinline__ int table_find(const int32_t* K, int32_t x) {
  constexpr int NB = SLOTS / 4;
  const int4* Kb = reinterpret_cast<const int4*>(K);
  const uint32_t b = hash_slot(x, __builtin_ctz(NB));
  return bucket_match<NB>(Kb, x, b, Kb[b]);
}

}  // namespace

// Looks x up in the bucket table: true when the lane is valid and x is in
// the table, with *off the byte offset inside the counter array C of x's
// slot (slot j of bucket b is counter 4b + j, at byte 16b + 4j). One 16-byte
// read unless x's home bucket is full and does not hold x (rare in a sparse
// table). The matching slot comes from four compares whose lane masks are
// combined on the scalar unit.
template <int NB>
__device__ __forceinline__ bool bucket_credit(const int4* Kb, int32_t x, bool valid, int* off) {
  uint32_t b = hash_slot(x, __builtin_ctz(NB));
  int4 q = Kb[b];
  bool e1 = q.y == x, e2 = q.z == x, e3 = q.w == x;
  bool hit = (q.x == x) | e1 | e2 | e3;
  int o = (int)(b << 4) + ((e1 | e3) ? 4 : 0) + ((e2 | e3) ? 8 : 0);
  bool more = valid & !hit & (q.w >= 0);
  while (more) {
    b = (b + 1) & (NB - 1);
    q = Kb[b];
    e1 = q.y == x;
    e2 = q.z == x;
    e3 = q.w == x;
    hit = (q.x == x) | e1 | e2 | e3;
    o = (int)(b << 4) + ((e1 | e3) ? 4 : 0) + ((e2 | e3) ? 8 : 0);
    more = !hit & (q.w >= 0);
  }
  *off = o;
  return valid & hit;
}

__device__ __forceinline__ void credit(uint32_t* C, int off) {
  atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(C) + off), 1u);
}

// Two-choice cuckoo table of SLOTS int32 keys (-1 = empty), one key per
// slot (Pagh and Rodler 2001; built in parallel with atomic exchanges as in
// Alcantara et al. 2009): key x sits in slot a(x) or b(x), so a lookup is two
// 4-byte LDS reads and two compares, with no probe loop. Ids share a slot
// pair when their low 24 bits agree.
template <int SLOTS>
__device__ __forceinline__ void cuckoo_pos(int32_t x, uint32_t* a, uint32_t* b) {
  constexpr int bits = __builtin_ctz(SLOTS);
  const uint32_t lo = (uint32_t)x & 0xFFFFFFu;
  *a = (lo * 0x9E3779u) >> (32 - bits);
  *b = (lo * 0x3C6EF3u) >> (32 - bits);
}

// The same two slots as byte offsets (4 x slot).
template <int SLOTS>
__device__ __forceinline__ void cuckoo_off(int32_t x, uint32_t* a, uint32_t* b) {
  cuckoo_pos<SLOTS>(x, a, b);
  *a <<= 2;
  *b <<= 2;
}

// Eviction chains longer than this give up: the caller then rebuilds the
// node's table in the bucket layout.
constexpr int kCuckooMaxChain = 48;

// Inserts x (absent from the table; keys are distinct). Each thread holds
// exactly one key outside the table at any time, so concurrent inserts lose
// nothing while they succeed. False: the chain gave up and the key it held
// is not in the table.
template <int SLOTS>
__device__ __forceinline__ bool cuckoo_insert(int32_t* K, int32_t x) {
  uint32_t a, b;
  cuckoo_pos<SLOTS>(x, &a, &b);
  if (atomicCAS(&K[a], -1, x) == -1 || atomicCAS(&K[b], -1, x) == -1) return true;
  uint32_t pos = a;
#pragma unroll 1
  for (int it = 0; it < kCuckooMaxChain; ++it) {
    x = atomicExch(&K[pos], x);
    if (x == -1) return true;
    cuckoo_pos<SLOTS>(x, &a, &b);  // the evicted key moves to its other slot
    pos = pos == a ? b : a;
  }
  return false;
}

// Slot of x in a complete cuckoo table, or -1.
template <int SLOTS>
__device__ __forceinline__ int cuckoo_find(const int32_t* K, int32_t x) {
  uint32_t a, b;
  cuckoo_pos<SLOTS>(x, &a, &b);
  return K[a] == x ? (int)a : K[b] == x ? (int)b : -1;
}

// Probes of the streaming loops: true when the lane is valid and x is in the
// table, with *off the byte offset of x's counter in C (4 x slot). The
// callers count the hits (per lane in a register on the long-list path, so
// that no scalar instruction is spent per 64 ids).
template <int NB>
struct BucketProbe {
  const int4* Kb;
  __device__ __forceinline__ bool operator()(int32_t x, bool valid, int* off) const {
    return bucket_credit<NB>(Kb, x, valid, off);
  }
};

template <int SLOTS>
struct CuckooProbe {
  const int32_t* K;
  __device__ __forceinline__ bool operator()(int32_t x, bool valid, int* off) const {
    x = valid ? x : -2;  // in no table
    uint32_t a, b;
    cuckoo_off<SLOTS>(x, &a, &b);
    const char* Kc = reinterpret_cast<const char*>(K);
    const bool ea = *reinterpret_cast<const int32_t*>(Kc + a) == x;
    const bool eb = *reinterpret_cast<const int32_t*>(Kc + b) == x;
    *off = (int)(ea ? a : b);
    return ea | eb;
  }
};

// Sum over the 64 lanes of a wavefront (all active): 16-lane row sums by
// DPP lane permutations (pairs, quads, half-row and row mirrors), then the
// four row sums read on the scalar unit.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xf, 0xf, false);  // row_half_mirror
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xf, 0xf, false);  // row_mirror
  return (uint32_t)(__builtin_amdgcn_readlane((int)x, 0) + __builtin_amdgcn_readlane((int)x, 16) +
                    __builtin_amdgcn_readlane((int)x, 32) + __builtin_amdgcn_readlane((int)x, 48));
}

// LDS of one node group of the wave-stream kernel.
template <int SLOTS, int CAP>
struct WaveGroupLds {
  int4 K[SLOTS / 4];     // bucket table of N+(u)
  uint32_t C[SLOTS];     // per-slot triangle credits
  int32_t Wb[CAP];       // N+(w) begins (offsets < 2^30)
  int32_t Wn[CAP];       // |N+(w)|
  int32_t Ws[CAP];       // slot of w
  uint32_t Wc[CAP];      // hits per streamed list (packed phase)
  int32_t Wl[CAP];       // indices of the lists streamed one by one
  int32_t nlong;         // number of such lists
  int32_t fail;          // a cuckoo insert gave up
};

// Lists shorter than this are streamed packed: a wavefront covers several
// short lists per step instead of one list per step.
constexpr int32_t kPackShort = 64;
// Steps of 64 ids whose gathers are issued together in the packed streams.
constexpr int kPackUnroll = 3;

// Lanes per node on the packed small-node path by default (d+ <= kSmallGS).
constexpr int kSmallGS = 16;

// Packed streaming of the short lists among items [i0, i1) of a group: a
// window of up to 64 lists sits in the lanes (begin, length, inclusive
// prefix of lengths); each step gives every lane one id of the window's
// concatenation, found by a shuffle binary search over the prefixes. A hit
// credits its table slot and its list's counter Wc. Returns the wave's hits.
template <typename Probe>
__device__ __forceinline__ uint32_t stream_packed(int32_t i0, int32_t i1, const int32_t* Wb, const int32_t* Wn,
                                                  uint32_t* Wc, const int32_t* __restrict__ dcol, Probe probe,
                                                  uint32_t* C) {
  const int lane = lane_id();
  uint32_t hits = 0;
  for (int32_t base = i0; base < i1; base += kWave) {
    const int32_t li = base + lane;
    int32_t nb = 0, bb = 0;
    if (li < i1) {
      nb = Wn[li];
      bb = Wb[li];
      if (nb >= kPackShort) nb = 0;  // long lists are streamed one by one
    }
    const int32_t incl = wave_incl_scan(nb);
    const int32_t total = __shfl(incl, kWave - 1, kWave);
    const int32_t dlt = bb - (incl - nb);  // list k's id at t: dcol[dlt_k + t]
    for (int32_t t0 = 0; t0 < total; t0 += kPackUnroll * kWave) {
      // kPackUnroll independent gathers in flight before the probes
      int32_t x[kPackUnroll];
      int kk[kPackUnroll];
#pragma unroll
      for (int r = 0; r < kPackUnroll; ++r) {
        const int32_t t = t0 + r * kWave + lane;
        int k = 0;
#pragma unroll
        for (int step = kWave / 2; step > 0; step >>= 1) {
          const int32_t v = __shfl(incl, k + step - 1, kWave);
          if (v <= t) k += step;
        }
        const int32_t at = __shfl(dlt, k, kWave) + t;
        x[r] = t < total ? dcol[at] : -1;
        kk[r] = k;
      }
#pragma unroll
      for (int r = 0; r < kPackUnroll; ++r) {
        if (t0 + r * kWave >= total) break;
        int off;
        const bool hit = probe(x[r], t0 + r * kWave + lane < total, &off);
        hits += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(hit));
        if (hit) {
          credit(C, off);
          atomicAdd(&Wc[base + kk[r]], 1u);
        }
      }
    }
  }
  return hits;
}

// U chunks of 64 ids of L[p..n) into x, through a raw buffer view of
// L[p..n): the offsets are lane * 4 + k * 256, which its range check covers
// exactly, so lanes past n read 0 without a memory access. All U loads are
// issued, which keeps the wait counts of the caller's pipeline exact.
template <int U>
__device__ __forceinline__ void load_chunk(int32_t (&x)[U], const int32_t* L, int32_t p, int32_t n, int lane) {
  static_assert(U * kWave * 4 <= 4096, "per-load offsets must fit the 12-bit immediate field");
  const int32_t left = n > p ? n - p : 0;
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(L + p), (short)0, left * 4, kRawBufferWord3);
#pragma unroll
  for (int k = 0; k < U; ++k) x[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4 + k * kWave * 4, 0, 0);
}

// One wavefront streams the long lists Wl[j] (j = j0, j0 + step, ... < nl)
// against the table, U loads of 64 ids per step: the next step's loads
// (same list, or the first chunk of the next one) are in flight while the
// current chunk is probed. Base and length of a list are wave-uniform
// (scalar registers). Each hit credits its table slot and the lane's hit
// count; at the end of a list the lanes' counts are summed (DPP) and
// done(i, hits) receives list i's hit count (wave-uniform). Per chunk of 64
// ids only the exit test and the credit's exec mask use the scalar unit.
// Returns the wave's hits.
template <int U, typename Probe, typename Done>
__device__ __forceinline__ uint32_t stream_long(int32_t j0, int32_t step, int32_t nl, const int32_t* Wl,
                                                const int32_t* Wb, const int32_t* Wn,
                                                const int32_t* __restrict__ dcol, Probe probe, uint32_t* C,
                                                Done done) {
  // j0 is the wave's index inside its group: uniform, but not provably so
  int32_t j = __builtin_amdgcn_readfirstlane(j0);
  if (j >= nl) return 0;
  const int lane = lane_id();
  int32_t i = __builtin_amdgcn_readfirstlane(Wl[j]);
  int32_t b = __builtin_amdgcn_readfirstlane(Wb[i]);
  int32_t n = __builtin_amdgcn_readfirstlane(Wn[i]);
  int32_t p = 0;
  uint32_t total = 0, hv = 0;  // hv: this lane's hits in list i
  // one pipeline step: load the chunk after (i, p) into nxt, probe cur;
  // false once the last list is done. Two register sets alternate, so no
  // copy has to wait for the loads in flight.
  auto advance = [&](int32_t (&cur)[U], int32_t (&nxt)[U]) -> bool {
    int32_t nj = j, ni = i, nb = b, nn = n, np = p + U * kWave;
    if (np >= n) {  // list i ends with this chunk
      nj = j + step;
      np = 0;
      nn = 0;
      if (nj < nl) {
        ni = __builtin_amdgcn_readfirstlane(Wl[nj]);
        nb = __builtin_amdgcn_readfirstlane(Wb[ni]);
        nn = __builtin_amdgcn_readfirstlane(Wn[ni]);
      }
    }
    load_chunk<U>(nxt, dcol + nb, np, nn, lane);
    const int32_t rem = n - p;  // ids of list i from p on
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (k * kWave >= rem) break;
      int off;
      const bool hit = probe(cur[k], lane + k * kWave < rem, &off);
      if (hit) credit(C, off);
      hv += (uint32_t)hit;
    }
    if (np == 0) {
      const uint32_t cw = wave_sum_u32(hv);
      hv = 0;
      done(i, cw);
      total += cw;
      if (nj >= nl) return false;
    }
    j = nj;
    i = ni;
    b = nb;
    n = nn;
    p = np;
    return true;
  };
  int32_t x[U], y[U];
  load_chunk<U>(x, dcol + b, 0, n, lane);
  while (advance(x, y) && advance(y, x)) {
  }
  return total;
}

// Builds the cuckoo table of the keys src[0..len) for a group of G lanes
// (g = lane in group). If an insert gives up, the table is rebuilt in the
// bucket layout instead. Returns true for a cuckoo table (group-uniform).
template <int G, int SLOTS, int CAP>
__device__ __forceinline__ bool build_cuckoo(WaveGroupLds<SLOTS, CAP>& S, const int32_t* __restrict__ src,
                                             int32_t len, int g) {
  int32_t* K = reinterpret_cast<int32_t*>(S.K);
  for (int i = g; i < len; i += G)
    if (!cuckoo_insert<SLOTS>(K, src[i])) S.fail = 1;
  group_sync<G>();
  if (__builtin_amdgcn_readfirstlane(S.fail) == 0) return true;
  for (int s = g; s < SLOTS; s += G) K[s] = -1;
  group_sync<G>();
  for (int i = g; i < len; i += G) bucket_insert<SLOTS / 4>(K, src[i]);
  group_sync<G>();
  return false;
}

// One node u (u < 0: inactive group) counted by a group of G lanes (G a
// multiple of 64; when G > 64 the group is the whole block).
// w_max > 0 (min-side mode): edges u->w with d+(u) < d+(w) <= w_max are left
// to w's in-list pass (node_count_inw), which then streams the shorter list.
// CK: N+(u) goes into a cuckoo table (bucket table if its build gives up).
template <int G, int SLOTS, int CAP, int U, bool CK = false>
__device__ __forceinline__ void node_count_wave(int32_t u, WaveGroupLds<SLOTS, CAP>& S,
                                                unsigned long long* red, const int64_t* __restrict__ doff,
                                                const int32_t* __restrict__ dcol,
                                                unsigned long long* __restrict__ T,
                                                unsigned long long* __restrict__ tot, int32_t w_max = 0) {
  static_assert(G % kWave == 0 && SLOTS % 4 == 0 && SLOTS >= 2 * CAP, "shape");
  constexpr int WPG = G / kWave;
  constexpr int NB = SLOTS / 4;
  const int g = threadIdx.x % G;
  const int wv = g / kWave;
  const int lane = lane_id();
  const bool active = u >= 0;
  int32_t* K = reinterpret_cast<int32_t*>(S.K);
  int64_t beg = 0;
  int32_t len = 0;  // an inactive group runs every phase with an empty list
  if (active) {
    beg = doff[u];
    len = (int32_t)(doff[u + 1] - beg);
  }
  for (int s = g; s < SLOTS; s += G) { K[s] = -1; S.C[s] = 0; }
  if (g == 0) { S.nlong = 0; S.fail = 0; }
  group_sync<G>();
  bool ck = false;
  if constexpr (CK) ck = build_cuckoo<G>(S, dcol + beg, len, g);
  for (int i = g; i < len; i += G) {
    const int32_t w = dcol[beg + i];
    if constexpr (CK) S.Ws[i] = ck ? cuckoo_find<SLOTS>(K, w) : table_find<SLOTS>(K, w);
    else S.Ws[i] = bucket_insert<NB>(K, w);
    const int64_t b = doff[w];
    int32_t wn = (int32_t)(doff[w + 1] - b);
    // edges u->w with d+(u) < d+(w) <= w_max are counted from w's in-list
    if (len < wn && wn <= w_max) wn = 0;
    S.Wb[i] = (int32_t)b;
    S.Wn[i] = wn;
    S.Wc[i] = 0;
    if (wn >= kPackShort) S.Wl[atomicAdd(&S.nlong, 1)] = i;
  }
  group_sync<G>();
  const int32_t nl = __builtin_amdgcn_readfirstlane(S.nlong);
  auto done = [&](int32_t i, uint32_t cw) {
    if (cw && lane == 0) atomicAdd(&S.C[S.Ws[i]], cw);
  };
  const int32_t p0 = wv * len / WPG, p1 = (wv + 1) * len / WPG;
  uint32_t tu;  // wave-uniform
  if (ck) {
    const CuckooProbe<SLOTS> probe{K};
    tu = stream_long<U>(wv, WPG, nl, S.Wl, S.Wb, S.Wn, dcol, probe, S.C, done);
    tu += stream_packed(p0, p1, S.Wb, S.Wn, S.Wc, dcol, probe, S.C);
  } else {
    const BucketProbe<NB> probe{S.K};
    tu = stream_long<U>(wv, WPG, nl, S.Wl, S.Wb, S.Wn, dcol, probe, S.C, done);
    tu += stream_packed(p0, p1, S.Wb, S.Wn, S.Wc, dcol, probe, S.C);
  }
  group_sync<G>();
  for (int i = g; i < len; i += G)
    if (S.Wc[i]) atomicAdd(&S.C[S.Ws[i]], S.Wc[i]);
  group_sync<G>();
  for (int s = g; s < SLOTS; s += G) {
    const int32_t k = K[s];
    const uint32_t c = S.C[s];
    if (k >= 0 && c) atomicAdd(&T[k], (unsigned long long)c);
  }
  if constexpr (WPG == 1) {
    if (active && lane == 0 && tu) {
      atomicAdd(&T[u], (unsigned long long)tu);
      credit_total(tot, tu);
    }
  } else {
    if (lane == 0) red[wv] = tu;
    __syncthreads();
    if (active && g == 0) {
      unsigned long long t = 0;
      for (int k = 0; k < WPG; ++k) t += red[k];
      if (t) atomicAdd(&T[u], t);
      credit_total(tot, t);
    }
    __syncthreads();  // red and the table may be reused by the caller
  }
}

// In-list side of the min-side split: a group owns node w and one chunk of
// at most CAP of its in-neighbours u (rank(u) < rank(w)). N+(w) is the LDS
// table; for every in-neighbour with 2 <= d+(u) < d+(w) one wavefront
// streams N+(u) against it. A hit x is the triangle u < w < x: x is credited
// in the table, w in the group total, u with one global atomic per in-edge.
template <int G, int SLOTS, int CAP, int U, bool CK = false>
__device__ __forceinline__ void node_count_inw(int32_t w, int64_t chunk, WaveGroupLds<SLOTS, CAP>& S,
                                               unsigned long long* red, const int64_t* __restrict__ doff,
                                               const int32_t* __restrict__ dcol,
                                               const int64_t* __restrict__ dinoff,
                                               const int32_t* __restrict__ dincol,
                                               unsigned long long* __restrict__ T,
                                               unsigned long long* __restrict__ tot) {
  constexpr int WPG = G / kWave;
  constexpr int NB = SLOTS / 4;
  const int g = threadIdx.x % G;
  const int wv = g / kWave;
  const int lane = lane_id();
  const bool active = w >= 0;
  int32_t* K = reinterpret_cast<int32_t*>(S.K);
  int64_t beg = 0, ib = 0;
  int32_t len = 0, nin = 0;
  if (active) {
    beg = doff[w];
    len = (int32_t)(doff[w + 1] - beg);
    ib = dinoff[w] + chunk * CAP;
    nin = (int32_t)min((int64_t)CAP, dinoff[w + 1] - ib);
  }
  for (int s = g; s < SLOTS; s += G) { K[s] = -1; S.C[s] = 0; }
  if (g == 0) { S.nlong = 0; S.fail = 0; }
  group_sync<G>();
  bool ck = false;
  if constexpr (CK) ck = build_cuckoo<G>(S, dcol + beg, len, g);
  else for (int i = g; i < len; i += G) bucket_insert<NB>(K, dcol[beg + i]);
  for (int i = g; i < nin; i += G) {
    const int32_t u = dincol[ib + i];
    const int64_t b = doff[u];
    int32_t nu = (int32_t)(doff[u + 1] - b);
    if (nu < 2 || nu >= len) nu = 0;
    S.Wb[i] = (int32_t)b;
    S.Wn[i] = nu;
    S.Ws[i] = u;
    S.Wc[i] = 0;
    if (nu >= kPackShort) S.Wl[atomicAdd(&S.nlong, 1)] = i;
  }
  group_sync<G>();
  const int32_t nl = __builtin_amdgcn_readfirstlane(S.nlong);
  auto done = [&](int32_t i, uint32_t cu) {
    if (cu && lane == 0) atomicAdd(&T[S.Ws[i]], (unsigned long long)cu);
  };
  const int32_t p0 = wv * nin / WPG, p1 = (wv + 1) * nin / WPG;
  uint32_t tw;  // wave-uniform
  if (ck) {
    const CuckooProbe<SLOTS> probe{K};
    tw = stream_long<U>(wv, WPG, nl, S.Wl, S.Wb, S.Wn, dcol, probe, S.C, done);
    tw += stream_packed(p0, p1, S.Wb, S.Wn, S.Wc, dcol, probe, S.C);
  } else {
    const BucketProbe<NB> probe{S.K};
    tw = stream_long<U>(wv, WPG, nl, S.Wl, S.Wb, S.Wn, dcol, probe, S.C, done);
    tw += stream_packed(p0, p1, S.Wb, S.Wn, S.Wc, dcol, probe, S.C);
  }
  group_sync<G>();
  for (int i = g; i < nin; i += G)
    if (S.Wc[i]) atomicAdd(&T[S.Ws[i]], (unsigned long long)S.Wc[i]);
  for (int s = g; s < SLOTS; s += G) {
    const int32_t k = K[s];
    const uint32_t c = S.C[s];
    if (k >= 0 && c) atomicAdd(&T[k], (unsigned long long)c);
  }
  if constexpr (WPG == 1) {
    if (active && lane == 0 && tw) {
      atomicAdd(&T[w], (unsigned long long)tw);
      credit_total(tot, tw);
    }
  } else {
    if (lane == 0) red[wv] = tw;
    __syncthreads();
    if (active && g == 0) {
      unsigned long long t = 0;
      for (int k = 0; k < WPG; ++k) t += red[k];
      if (t) atomicAdd(&T[w], t);
      credit_total(tot, t);
    }
    __syncthreads();
  }
}

// One bin in min-side mode: the first ceil(nu/GPB) blocks count the bin's
// nodes from their out-lists (skipping edges owned by in-lists), the rest run
// the bin's in-list chunks. In-list items: the nodes inl[0..nin) with chunk
// prefix inc[0..nin] (inc[0] need not be 0).
// owner[j] - base = p, the index of item j's node in list: the chunk -> owner
// map built with the chunk prefix.
struct InItems {
  const int32_t* list;
  const int64_t* coff;
  const int32_t* owner;
  int32_t base;
  int32_t nodes;
  int64_t items;
};

// In-list item j of a bin: its owner w and chunk (w = -1 past the items).
__device__ __forceinline__ void in_item(const InItems& in, int64_t j, int32_t* w, int64_t* chunk) {
  *w = -1;
  *chunk = 0;
  if (j >= in.items) return;
  const int32_t p = in.owner[j] - in.base;
  *w = in.list[p];
  *chunk = in.coff[0] + j - in.coff[p];
}

template <int NT, int G, int SLOTS, int CAP, int U, bool CK>
__global__ __launch_bounds__(NT) void k_count_ms(const int32_t* __restrict__ list, int32_t nlist, InItems in,
                                                 int32_t w_max, const int64_t* __restrict__ doff,
                                                 const int32_t* __restrict__ dcol,
                                                 const int64_t* __restrict__ dinoff,
                                                 const int32_t* __restrict__ dincol,
                                                 unsigned long long* __restrict__ T,
                                                 unsigned long long* __restrict__ tot) {
  static_assert(NT % G == 0 && (G == kWave || G == NT), "groups are single waves or whole blocks");
  constexpr int GPB = NT / G;
  __shared__ WaveGroupLds<SLOTS, CAP> lds[GPB];
  __shared__ unsigned long long red[NT / kWave];
  const int gi = threadIdx.x / G;
  const int64_t nbu = ((int64_t)nlist + GPB - 1) / GPB;
  if ((int64_t)blockIdx.x < nbu) {
    const int64_t idx = (int64_t)blockIdx.x * GPB + gi;
    node_count_wave<G, SLOTS, CAP, U, CK>(idx < nlist ? list[idx] : -1, lds[gi], red, doff, dcol, T, tot, w_max);
    return;
  }
  int32_t w;
  int64_t chunk;
  in_item(in, ((int64_t)blockIdx.x - nbu) * GPB + gi, &w, &chunk);
  node_count_inw<G, SLOTS, CAP, U, CK>(w, chunk, lds[gi], red, doff, dcol, dinoff, dincol, T, tot);
}

// Merge variant for short lists: a group of G lanes owns node u and each
// lane takes whole out-edges u->w, merging the sorted lists N+(u) and N+(w)
// straight from memory (the classic two-pointer intersection; N+(u) is
// re-read by every lane of the group, from cache). Hits go to T with global
// atomics, which suits graphs with few triangles per edge.
template <int G>
__device__ __forceinline__ void node_count_merge(int32_t u, const int64_t* __restrict__ doff,
                                                 const int32_t* __restrict__ dcol,
                                                 unsigned long long* __restrict__ T,
                                                 unsigned long long* __restrict__ tot) {
  const int g = threadIdx.x % G;
  unsigned long long tu = 0;
  if (u >= 0) {
    const int64_t ub = doff[u];
    const int32_t nu = (int32_t)(doff[u + 1] - ub);
    const int32_t* U = dcol + ub;
    for (int32_t i = g; i < nu; i += G) {
      const int32_t w = U[i];
      const int64_t wb = doff[w];
      const int32_t nw = (int32_t)(doff[w + 1] - wb);
      const int32_t* W = dcol + wb;
      int32_t a = 0, b = 0;
      uint32_t c = 0;
      int32_t xa = nu > 0 ? U[0] : 0, xb = nw > 0 ? W[0] : 0;
      while (a < nu && b < nw) {
        if (xa == xb) {
          atomicAdd(&T[xa], 1ull);
          ++c;
          ++a;
          ++b;
          xa = a < nu ? U[a] : 0;
          xb = b < nw ? W[b] : 0;
        } else if (xa < xb) {
          ++a;
          xa = a < nu ? U[a] : 0;
        } else {
          ++b;
          xb = b < nw ? W[b] : 0;
        }
      }
      if (c) atomicAdd(&T[w], (unsigned long long)c);
      tu += c;
    }
  }
  tu = group_sum<unsigned long long, G>(tu);
  if (u >= 0 && g == 0 && tu) {
    atomicAdd(&T[u], tu);
    credit_total(tot, tu);
  }
}

// Fallback for out-lists of any length: one block of 256 per node, N+(u)
// stays in global memory and is binary-searched; hits are credited with
// global atomics.
__device__ __forceinline__ void node_count_global(int32_t u, unsigned long long* red,
                                                  const int64_t* __restrict__ doff,
                                                  const int32_t* __restrict__ dcol,
                                                  unsigned long long* __restrict__ T,
                                                  unsigned long long* __restrict__ tot) {
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
  if (threadIdx.x == 0 && t) {
    atomicAdd(&T[u], t);
    credit_total(tot, t);
  }
}

__global__ __launch_bounds__(256) void k_count_global(const int32_t* __restrict__ list, int32_t nlist,
                                                      const int64_t* __restrict__ doff,
                                                      const int32_t* __restrict__ dcol,
                                                      unsigned long long* __restrict__ T,
                                                      unsigned long long* __restrict__ tot) {
  __shared__ unsigned long long red[256 / kWave];
  node_count_global(list[blockIdx.x], red, doff, dcol, T, tot);
}

// Hub variant: N+(u) as a bitmap over all node ids, one private bitmap per
// block in global memory (2 MB at 16.7M ids, L2-resident). The block sets
// u's bits, makes them visible (device fence, so that no stale L1 line
// survives), streams every N+(w) with its wavefronts (buffer loads, then one
// 4-byte bitmap load per id), credits x with a global atomic per hit and w
// once per list, and finally clears exactly the words it set, so the map is
// all zero again for the next node or launch. The grid never exceeds the
// number of bitmaps.
constexpr int kHubNT = 1024;

template <int U>
__global__ __launch_bounds__(kHubNT) void k_count_bitmap(const int32_t* __restrict__ list, int32_t nlist,
                                                         uint32_t* __restrict__ hubmap, int64_t map_words,
                                                         const int64_t* __restrict__ doff,
                                                         const int32_t* __restrict__ dcol,
                                                         unsigned long long* __restrict__ T,
                                                         unsigned long long* __restrict__ tot) {
  static_assert(U * kWave * 4 <= 4096, "per-load offsets must fit the 12-bit immediate field");
  constexpr int WPB = kHubNT / kWave;
  __shared__ unsigned long long red[WPB];
  uint32_t* map = hubmap + (int64_t)blockIdx.x * map_words;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  for (int32_t idx = blockIdx.x; idx < nlist; idx += gridDim.x) {
    const int32_t u = list[idx];
    const int64_t ub = doff[u];
    const int32_t nu = (int32_t)(doff[u + 1] - ub);
    for (int32_t i = threadIdx.x; i < nu; i += kHubNT) {
      const int32_t x = dcol[ub + i];
      atomicOr(&map[x >> 5], 1u << (x & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    unsigned long long tu = 0;
    for (int32_t i = __builtin_amdgcn_readfirstlane(wv); i < nu; i += WPB) {
      const int32_t w = __builtin_amdgcn_readfirstlane(dcol[ub + i]);
      const int64_t wb = doff[w];  // w is uniform, so are its bounds
      const int32_t wn = (int32_t)(doff[w + 1] - wb);
      uint32_t cw = 0;
      for (int32_t p = 0; p < wn; p += U * kWave) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(dcol + wb + p), (short)0, (wn - p) * 4,
                                              kRawBufferWord3);
        int32_t x[U];
#pragma unroll
        for (int k = 0; k < U; ++k) x[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4 + k * kWave * 4, 0, 0);
        uint32_t mw[U];
#pragma unroll
        for (int k = 0; k < U; ++k) mw[k] = p + k * kWave + lane < wn ? map[x[k] >> 5] : 0u;
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const bool hit = (mw[k] >> (x[k] & 31)) & 1u;
          cw += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(hit));
          if (hit) atomicAdd(&T[x[k]], 1ull);
        }
      }
      if (lane == 0) {
        if (cw) atomicAdd(&T[w], (unsigned long long)cw);
        tu += cw;  // cw is wave-uniform: counted once per wave for the block sum
      }
    }
    const unsigned long long t = block_sum<unsigned long long, kHubNT>(tu, red);
    if (threadIdx.x == 0 && t) {
      atomicAdd(&T[u], t);
      credit_total(tot, t);
    }
    __syncthreads();  // every probe of this node is done
    for (int32_t i = threadIdx.x; i < nu; i += kHubNT) map[dcol[ub + i] >> 5] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Several short-list nodes per wavefront: GS lanes per node (d+(u) <= GS),
// 64 / GS nodes per wave. Lane j of a node's lanes owns the out-edge to the
// j-th entry w of N+(u); each node has a bucket table of 4 * GS slots in
// LDS. The 64 lanes' lists N+(w) are streamed packed (one id per lane per
// step, its list found by a shuffle binary search over the lanes' length
// prefix) and each id is probed against the table of its list's node, so a
// wave keeps 64 independent loads in flight instead of walking dependent
// merge chains. Credits: x per table slot, w per list, u per node.
template <int GS>
struct SmallLds {
  int4 K[kWave / GS][GS];          // GS buckets (4 * GS slots) per node
  uint32_t C[kWave / GS][4 * GS];  // per-slot credits
  uint32_t Wc[kWave];              // hits per lane's list
};

// The packed stream of the small-node path: the 64 lanes' lists (begin wb,
// inclusive prefix incl of their lengths, total) against the lanes' node
// tables; a hit credits its table slot and its list's counter Wc.
template <int GS, bool CK>
__device__ __forceinline__ void small_stream(SmallLds<GS>& S, int32_t incl, int32_t total, int32_t excl, int32_t wb,
                                             const int32_t* __restrict__ dcol, int lane) {
  const int32_t dlt = wb - excl;  // list k's id at t: dcol[dlt_k + t]
  for (int32_t t0 = 0; t0 < total; t0 += kPackUnroll * kWave) {
    // kPackUnroll independent gathers in flight before the probes
    int32_t x[kPackUnroll];
    int kk[kPackUnroll];
#pragma unroll
    for (int r = 0; r < kPackUnroll; ++r) {
      const int32_t t = t0 + r * kWave + lane;
      int k = 0;
#pragma unroll
      for (int step = kWave / 2; step > 0; step >>= 1) {
        const int32_t v = __shfl(incl, k + step - 1, kWave);
        if (v <= t) k += step;
      }
      const int32_t at = __shfl(dlt, k, kWave) + t;
      x[r] = t < total ? dcol[at] : -1;
      kk[r] = k;
    }
#pragma unroll
    for (int r = 0; r < kPackUnroll; ++r) {
      if (t0 + r * kWave >= total) break;
      int off;
      bool hit;
      if constexpr (CK) {
        hit = CuckooProbe<4 * GS>{reinterpret_cast<const int32_t*>(S.K[kk[r] / GS])}(
            x[r], t0 + r * kWave + lane < total, &off);
      } else {
        hit = bucket_credit<GS>(S.K[kk[r] / GS], x[r], t0 + r * kWave + lane < total, &off);
      }
      if (hit) {
        credit(S.C[kk[r] / GS], off);
        atomicAdd(&S.Wc[kk[r]], 1u);
      }
    }
  }
}

// CK: the node tables are cuckoo tables (all of the wave's tables are
// rebuilt in the bucket layout if one insert gives up).
// Nodes with d+(u) > GS are left out; the returned lane mask has bit k * GS
// set for each such node list[first + k] (wave-uniform). w_max > 0
// (min-side mode): edges u->w with d+(u) < d+(w) <= w_max are left to w's
// in-list pass, as in node_count_wave.
template <int GS, bool CK = false>
__device__ __forceinline__ uint64_t nodes_count_small(const int32_t* __restrict__ list, int64_t first,
                                                      int64_t nlist, SmallLds<GS>& S,
                                                      const int64_t* __restrict__ doff,
                                                      const int32_t* __restrict__ dcol,
                                                      unsigned long long* __restrict__ T,
                                                      unsigned long long* __restrict__ tot, int32_t w_max = 0) {
  static_assert(kWave % GS == 0 && GS >= 4, "GS divides the wave");
  constexpr int NB = GS;
  const int lane = lane_id();
  const int nd = lane / GS, j = lane % GS;
  int32_t* K = reinterpret_cast<int32_t*>(S.K[nd]);
  uint32_t* C = S.C[nd];
  for (int s = j; s < 4 * GS; s += GS) {
    K[s] = -1;
    C[s] = 0;
  }
  S.Wc[lane] = 0;
  const int64_t idx = first + nd;
  int32_t u = -1, nu = 0, w = -1, wb = 0, wn = 0;
  int64_t ub = 0;
  if (idx < nlist) {
    u = list[idx];
    ub = doff[u];
    nu = (int32_t)(doff[u + 1] - ub);
  }
  const uint64_t big = __builtin_amdgcn_ballot_w64(j == 0 && nu > GS);
  if (nu > GS) {  // left to the caller
    u = -1;
    nu = 0;
  }
  wave_sync();
  bool gave_up = false;
  if (j < nu) {
    w = dcol[ub + j];
    if constexpr (CK) gave_up = !cuckoo_insert<4 * GS>(K, w);
    else bucket_insert<NB>(K, w);
    const int64_t b = doff[w];
    wb = (int32_t)b;
    wn = (int32_t)(doff[w + 1] - b);
    // edges u->w with d+(u) < d+(w) <= w_max are counted from w's in-list
    if (nu < wn && wn <= w_max) wn = 0;
  }
  wave_sync();
  bool ck = false;
  if constexpr (CK) {
    ck = __builtin_amdgcn_ballot_w64(gave_up) == 0;
    if (!ck) {
      for (int s = j; s < 4 * GS; s += GS) K[s] = -1;
      wave_sync();
      if (j < nu) bucket_insert<NB>(K, w);
      wave_sync();
    }
  }
  const int32_t incl = wave_incl_scan(wn);
  const int32_t total = __shfl(incl, kWave - 1, kWave);
  const int32_t excl = incl - wn;
  if (ck) small_stream<GS, true>(S, incl, total, excl, wb, dcol, lane);
  else small_stream<GS, false>(S, incl, total, excl, wb, dcol, lane);
  wave_sync();
  const uint32_t c = S.Wc[lane];
  if (c) atomicAdd(&T[w], (unsigned long long)c);
  const uint32_t tu = group_sum<uint32_t, GS>(c);
  if (j == 0 && tu) atomicAdd(&T[u], (unsigned long long)tu);
  const uint32_t tw = group_sum<uint32_t, kWave>(c);  // the wave's nodes together
  if (lane == 0) credit_total(tot, tw);
  for (int s = j; s < 4 * GS; s += GS) {
    const int32_t key = K[s];
    const uint32_t cs = C[s];
    if (key >= 0 && cs) atomicAdd(&T[key], (unsigned long long)cs);
  }
  return big;
}

// Bin kernel for short out-lists (d+ <= CAP <= 64), one wavefront per group:
// each wavefront takes 64 / GS consecutive nodes of the bin, counts those
// with d+ <= GS together on the packed small-node path, then the others one
// by one as node_count_wave does. The in-list side (blocks after the first
// ceil(nlist / (GPB * 64 / GS))) is k_count_ms's.
template <int NT, int SLOTS, int CAP, int U, bool CK, int GS>
__global__ __launch_bounds__(NT) void k_count_mss(const int32_t* __restrict__ list, int32_t nlist, InItems in,
                                                  int32_t w_max, const int64_t* __restrict__ doff,
                                                  const int32_t* __restrict__ dcol,
                                                  const int64_t* __restrict__ dinoff,
                                                  const int32_t* __restrict__ dincol,
                                                  unsigned long long* __restrict__ T,
                                                  unsigned long long* __restrict__ tot) {
  constexpr int GPB = NT / kWave;
  constexpr int NPW = kWave / GS;
  using WL = WaveGroupLds<SLOTS, CAP>;
  static_assert(CAP <= kWave && sizeof(SmallLds<GS>) <= sizeof(WL), "one wave's LDS holds either path");
  __shared__ WL lds[GPB];
  __shared__ unsigned long long red[GPB];
  const int gi = threadIdx.x / kWave;
  const int64_t nbu = ((int64_t)nlist + GPB * NPW - 1) / (GPB * NPW);
  if ((int64_t)blockIdx.x < nbu) {
    const int64_t first = ((int64_t)blockIdx.x * GPB + gi) * NPW;
    uint64_t big = nodes_count_small<GS, CK>(list, first, nlist, *reinterpret_cast<SmallLds<GS>*>(&lds[gi]), doff,
                                             dcol, T, tot, w_max);
    wave_sync();  // the small path's LDS is reused below
    while (big) {
      const int k = __builtin_ctzll(big) / GS;
      big &= big - 1;
      node_count_wave<kWave, SLOTS, CAP, U, CK>(list[first + k], lds[gi], red, doff, dcol, T, tot, w_max);
    }
    return;
  }
  int32_t w;
  int64_t chunk;
  in_item(in, ((int64_t)blockIdx.x - nbu) * GPB + gi, &w, &chunk);
  node_count_inw<kWave, SLOTS, CAP, U, CK>(w, chunk, lds[gi], red, doff, dcol, dinoff, dincol, T, tot);
}

// Persistent form (batched graphs): one launch covers every node of the
// DAG, in two phases.
// Phase 1, whole blocks: nodes above the block table's capacity (global
// fallback), then nodes for a whole block (d+ <= CB), one per pull from
// queue[0].
// Phase 2, single wavefronts on their own (no block barrier): single-wave
// nodes (d+ <= CW), then groups of short-list nodes: 8 at a time for the
// 8-lane merge (SMALL == 0) or 64 / SMALL at a time on the packed
// small-node path with SMALL lanes per node (d+ <= SMALL). A wave takes
// kPersistGrab items per atomic and issues its next grab before running the
// current items, so the atomic's latency hides behind their loads. Each wave
// owns a private LDS region in phase 2.
// Phase 2 is split into kPersistSegs segments of consecutive graphs (equal
// shares of the edges), one per XCD: the chip hands out blocks to its XCDs
// in turn, so block b starts on segment b mod kPersistSegs and the graphs a
// segment holds stay in one XCD's L2 while they are counted; a wave whose
// segment is empty takes items of the next ones.
constexpr int kPersistGrab = 8;

template <int SW, int CW, int SB, int CB, int SMALL = 0, bool CK = false>
__global__ __launch_bounds__(256) void k_count_persist(const int32_t* __restrict__ glist, int32_t ng,
                                                       const int32_t* __restrict__ blist, int32_t nbk,
                                                       const int32_t* __restrict__ wlist,
                                                       const int32_t* __restrict__ mlist,
                                                       const int32_t* __restrict__ seg,
                                                       int32_t* __restrict__ queue,
                                                       const int64_t* __restrict__ doff,
                                                       const int32_t* __restrict__ dcol,
                                                       unsigned long long* __restrict__ T,
                                                       unsigned long long* __restrict__ tot) {
  using BL = WaveGroupLds<SB, CB>;
  using WL = WaveGroupLds<SW, CW>;
  constexpr int kGS = SMALL ? SMALL : kSmallGS;
  using SL = SmallLds<kGS>;
  constexpr size_t kWaveBytes = ((sizeof(WL) > sizeof(SL) ? sizeof(WL) : sizeof(SL)) + 15) / 16 * 16;
  constexpr size_t kBytes = sizeof(BL) > 4 * kWaveBytes ? sizeof(BL) : 4 * kWaveBytes;
  __shared__ __align__(16) unsigned char smem[kBytes];
  __shared__ unsigned long long red[256 / kWave];
  __shared__ int32_t chunk;
  const int32_t n1 = ng + nbk;
  while (true) {
    if (threadIdx.x == 0) chunk = atomicAdd(queue, 1);
    __syncthreads();
    const int32_t c = chunk;
    __syncthreads();
    if (c >= n1) break;
    if (c < ng) node_count_global(glist[c], red, doff, dcol, T, tot);
    else node_count_wave<256, SB, CB, 4, CK>(blist[c - ng], *reinterpret_cast<BL*>(smem), red, doff, dcol, T, tot);
    __syncthreads();
  }
  constexpr int NPW = SMALL ? kWave / kGS : kWave / 8;  // short-list nodes per wave item
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  unsigned char* mine = smem + wv * kWaveBytes;
  // Phase 2 takes the items of segment x = (this block's XCD) first, then
  // moves on to the other segments once it is empty: seg[x .. x+1] bound the
  // segment's single-wave nodes in wlist, seg[kPersistSegs + 1 + x ..] its
  // short-list nodes in mlist; queue[2 + x] counts the items taken.
  const int x0 = (int)(blockIdx.x % kPersistSegs);
  for (int t = 0; t < kPersistSegs; ++t) {
    const int x = (x0 + t) % kPersistSegs;
    const int32_t wb = seg[x], nwx = seg[x + 1] - wb;
    const int32_t mb = seg[kPersistSegs + 1 + x], me = seg[kPersistSegs + 2 + x];
    const int32_t n2 = nwx + (int32_t)(((int64_t)(me - mb) + NPW - 1) / NPW);
    int32_t got = 0;
    if (lane == 0) got = atomicAdd(queue + 2 + x, kPersistGrab);
    int32_t cur = __builtin_amdgcn_readfirstlane(got);
    while (cur < n2) {
      int32_t nxt = 0;
      if (lane == 0) nxt = atomicAdd(queue + 2 + x, kPersistGrab);
      const int32_t end = min(cur + kPersistGrab, n2);
      for (int32_t it = cur; it < end; ++it) {
        if (it < nwx) {
          node_count_wave<kWave, SW, CW, 4, CK>(wlist[wb + it], *reinterpret_cast<WL*>(mine), red, doff, dcol, T,
                                                tot);
        } else if constexpr (SMALL != 0) {
          nodes_count_small<kGS, CK>(mlist, mb + (int64_t)(it - nwx) * NPW, me, *reinterpret_cast<SL*>(mine), doff,
                                     dcol, T, tot);
        } else {
          const int64_t k = mb + (int64_t)(it - nwx) * NPW + lane / 8;
          node_count_merge<8>(k < me ? mlist[k] : -1, doff, dcol, T, tot);
        }
      }
      cur = __builtin_amdgcn_readlane(nxt, 0);
    }
  }
}

// Segment bounds of the persistent kernel's phase 2 (see k_count_persist):
// for x = 0 .. kPersistSegs, out[x] = first index of wlist whose node is at
// least thr[x], out[kPersistSegs + 1 + x] the same in mlist. The lists are in
// ascending node order up to the classification's blocks of ids, so a
// boundary may land inside one such block: locality only, every item is
// still taken exactly once.
__global__ void k_persist_segments(const int32_t* __restrict__ wlist, int32_t nw, const int32_t* __restrict__ mlist,
                                   int32_t nm, const int64_t* __restrict__ thr, int32_t* __restrict__ out) {
  const int i = threadIdx.x;
  if (i >= 2 * (kPersistSegs + 1)) return;
  const bool m = i > kPersistSegs;
  const int x = m ? i - kPersistSegs - 1 : i;
  const int32_t* L = m ? mlist : wlist;
  const int32_t n = m ? nm : nw;
  int32_t r;
  if (x == 0) r = 0;
  else if (x == kPersistSegs) r = n;
  else {
    const int64_t t = thr[x];
    int32_t lo = 0, hi = n;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if ((int64_t)L[mid] < t) lo = mid + 1; else hi = mid;
    }
    r = lo;
  }
  out[i] = r;
}

hipError_t launch_persist_segments(const int32_t* wlist, int32_t nw, const int32_t* mlist, int32_t nm,
                                   const int64_t* thr, int32_t* out, hipStream_t s) {
  k_persist_segments<<<1, 64, 0, s>>>(wlist, nw, mlist, nm, thr, out);
  return hipGetLastError();
}

struct PersistShape { int sw, cw, sb, cb, small, ck = 0; };
static constexpr PersistShape kPersist[] = {
    {256, 64, 1024, 256, 0},   // 0: block nodes up to d+ 256, 8-lane merge
    {256, 64, 4096, 1024, 0},  // 1: block nodes up to d+ 1024, 8-lane merge
    {256, 64, 1024, 256, 16},  // 2: as 0, short lists on the packed small-node path (16 lanes per node)
    {256, 64, 4096, 1024, 16}, // 3: as 1, short lists on the packed small-node path
    {256, 64, 1024, 256, 32},  // 4: as 2 with 32 lanes per node (d+ <= 32)
    {256, 64, 1024, 256, 8},   // 5: as 2 with 8 lanes per node (d+ <= 8)
    {256, 64, 1024, 256, 16, 1},   // 6: as 2 with cuckoo tables (bucket tables where a build gives up)
    {256, 64, 4096, 1024, 16, 1},  // 7: as 3 with cuckoo tables
};
int persist_variant_count() { return (int)(sizeof(kPersist) / sizeof(kPersist[0])); }
int persist_wave_cap(int v) { return kPersist[v].cw; }
int persist_block_cap(int v) { return kPersist[v].cb; }
int persist_merge_cap(int v) { return kPersist[v].small ? kPersist[v].small : kPersist[v].cw; }

const void* persist_kernel(int v) {
  switch (v) {
    case 0: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 1024, 256>);
    case 1: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 4096, 1024>);
    case 2: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 1024, 256, 16>);
    case 3: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 4096, 1024, 16>);
    case 4: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 1024, 256, 32>);
    case 5: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 1024, 256, 8>);
    case 6: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 1024, 256, 16, true>);
    case 7: return reinterpret_cast<const void*>(&k_count_persist<256, 64, 4096, 1024, 16, true>);
    default: return nullptr;
  }
}

template <int SW, int CW, int SB, int CB, int SMALL = 0, bool CK = false>
static void launch_persist(unsigned grid, const int32_t* glist, int32_t ng, const int32_t* blist, int32_t nbk,
                           const int32_t* wlist, const int32_t* mlist, const int32_t* seg, int32_t* queue,
                           const int64_t* doff, const int32_t* dcol, unsigned long long* T, unsigned long long* tot,
                           hipStream_t s) {
  k_count_persist<SW, CW, SB, CB, SMALL, CK><<<grid, 256, 0, s>>>(glist, ng, blist, nbk, wlist, mlist, seg, queue,
                                                                   doff, dcol, T, tot);
}

hipError_t launch_count_persist(int v, unsigned grid, const int32_t* glist, int32_t ng, const int32_t* blist,
                                int32_t nbk, const int32_t* wlist, const int32_t* mlist, const int32_t* seg,
                                int32_t* queue, const int64_t* doff, const int32_t* dcol, unsigned long long* T,
                                unsigned long long* tot, hipStream_t s) {
#define TRICC_PERSIST_ARGS grid, glist, ng, blist, nbk, wlist, mlist, seg, queue, doff, dcol, T, tot, s
  switch (v) {
    case 0: launch_persist<256, 64, 1024, 256>(TRICC_PERSIST_ARGS); break;
    case 1: launch_persist<256, 64, 4096, 1024>(TRICC_PERSIST_ARGS); break;
    case 2: launch_persist<256, 64, 1024, 256, 16>(TRICC_PERSIST_ARGS); break;
    case 3: launch_persist<256, 64, 4096, 1024, 16>(TRICC_PERSIST_ARGS); break;
    case 4: launch_persist<256, 64, 1024, 256, 32>(TRICC_PERSIST_ARGS); break;
    case 5: launch_persist<256, 64, 1024, 256, 8>(TRICC_PERSIST_ARGS); break;
    case 6: launch_persist<256, 64, 1024, 256, 16, true>(TRICC_PERSIST_ARGS); break;
    case 7: launch_persist<256, 64, 4096, 1024, 16, true>(TRICC_PERSIST_ARGS); break;
    default: return hipErrorInvalidValue;
  }
#undef TRICC_PERSIST_ARGS
  return hipGetLastError();
}

// Clears T[n], the kTotSlots total counters and the work-queue counters
// (phase 1 and one per phase-2 segment; a kernel, so that it can sit in a
// captured graph).
__global__ __launch_bounds__(256) void k_batch_zero(unsigned long long* __restrict__ T, int64_t n,
                                                    unsigned long long* __restrict__ tot,
                                                    int32_t* __restrict__ queue) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 < 2 + kPersistSegs) queue[i0] = 0;
  if (i0 < kTotSlots) tot[i0] = 0ull;
  for (int64_t i = i0; i < n; i += stride) T[i] = 0ull;
}

hipError_t launch_batch_zero(unsigned long long* T, int64_t n, unsigned long long* tot, int32_t* queue,
                             hipStream_t s) {
  int64_t g = (std::max<int64_t>(n, kTotSlots) + 255) / 256;
  if (g > 65536) g = 65536;
  k_batch_zero<<<(unsigned)g, 256, 0, s>>>(T, n, tot, queue);
  return hipGetLastError();
}

// Sum of the kTotSlots total counters by one block (fixed order).
__device__ __forceinline__ unsigned long long sum_total(const unsigned long long* __restrict__ tot,
                                                        unsigned long long* red) {
  unsigned long long acc = 0;
  for (int i = threadIdx.x; i < kTotSlots; i += 256) acc += tot[i];
  return block_sum<unsigned long long, 256>(acc, red);
}

// Per-graph epilogue: one block per graph g owns nodes [node_off[g],
// node_off[g+1]): CC(v) as in the single-graph epilogue, the graph's
// triangle total (sum of T / 3) and its average CC over its n_g nodes, each
// summed in a fixed order that depends only on the graph. Block 0 also
// writes the batch's total from the counters the intersection kernels fed
// (independent of T) to *batch_tri, if that is not null.
__global__ __launch_bounds__(256) void k_graph_epilogue(const int64_t* __restrict__ node_off,
                                                        const unsigned long long* __restrict__ T,
                                                        const int32_t* __restrict__ deg, float* __restrict__ cc,
                                                        unsigned long long* __restrict__ graph_tri,
                                                        double* __restrict__ graph_avg,
                                                        const unsigned long long* __restrict__ tot,
                                                        unsigned long long* __restrict__ batch_tri) {
  __shared__ double red_d[256 / kWave];
  __shared__ unsigned long long red_t[256 / kWave];
  const int64_t nb = node_off[blockIdx.x], ne = node_off[blockIdx.x + 1];
  double acc = 0.0;
  unsigned long long tacc = 0;
  for (int64_t v = nb + threadIdx.x; v < ne; v += 256) {
    const unsigned long long t = T[v];
    const int64_t d = deg[v];
    double r = 0.0;
    if (d >= 2) r = (2.0 * (double)t) / ((double)d * (double)(d - 1));
    cc[v] = (float)r;
    acc += r;
    tacc += t;
  }
  const double sd = block_sum<double, 256>(acc, red_d);
  const unsigned long long st = block_sum<unsigned long long, 256>(tacc, red_t);
  if (threadIdx.x == 0) {
    graph_tri[blockIdx.x] = st / 3ull;
    graph_avg[blockIdx.x] = ne > nb ? sd / (double)(ne - nb) : 0.0;
  }
  if (blockIdx.x == 0 && batch_tri) {
    const unsigned long long all = sum_total(tot, red_t);
    if (threadIdx.x == 0) *batch_tri = all;
  }
}

hipError_t launch_graph_epilogue(int32_t num_graphs, const int64_t* node_off, const unsigned long long* T,
                                 const int32_t* deg, float* cc, unsigned long long* graph_tri, double* graph_avg,
                                 const unsigned long long* tot, unsigned long long* batch_tri, hipStream_t s) {
  if (num_graphs <= 0) return hipSuccess;
  k_graph_epilogue<<<num_graphs, 256, 0, s>>>(node_off, T, deg, cc, graph_tri, graph_avg, tot, batch_tri);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Variant table. Every table variant is a min-side kernel (out-list side and
// in-list side of a bin); cap = the largest d+(u) its LDS table takes.
struct VariantInfo { int nt, g, slots, cap; };
static constexpr VariantInfo kVariants[] = {
    // bucket tables
    {256, 64, 128, 16},       // 0: d+ <= 16
    {256, 64, 256, 64},       // 1: d+ <= 64
    {256, 256, 1024, 256},    // 2: d+ <= 256
    {512, 512, 4096, 1024},   // 3: d+ <= 1024
    {1024, 1024, 8192, 4096}, // 4: d+ <= 4096
    {512, 512, 2048, 1024},   // 5: d+ <= 1024, denser table
    {512, 512, 4096, 2048},   // 6: d+ <= 2048
    {256, 256, 512, 256},     // 7: d+ <= 256, denser table
    // table-free kernels for any d+
    {256, 256, 0, 0x7fffffff},    // 8: global fallback (binary search of N+(u) in HBM)
    {1024, 1024, 0, 0x7fffffff},  // 9: hub bitmap in global memory
    // cuckoo tables (bucket tables where a build gives up)
    {256, 64, 128, 16},       // 10: d+ <= 16
    {256, 64, 256, 64},       // 11: d+ <= 64
    {256, 256, 1024, 256},    // 12: d+ <= 256
    {512, 512, 4096, 1024},   // 13: d+ <= 1024
    {1024, 1024, 8192, 4096}, // 14: d+ <= 4096
    {512, 512, 2048, 1024},   // 15: d+ <= 1024, denser table
    {512, 512, 4096, 2048},   // 16: d+ <= 2048
    {256, 256, 512, 256},     // 17: d+ <= 256, denser table
    {128, 128, 512, 128},     // 18: d+ <= 128, two wavefronts per node
    {128, 128, 1024, 256},    // 19: d+ <= 256, two wavefronts per node
    {1024, 1024, 4096, 2048}, // 20: d+ <= 2048, sixteen wavefronts per node (two blocks per CU
                              //     fill its wave slots, against 16 waves for variant 16)
    // short out-lists: four nodes with d+ <= 16 per wavefront, the rest as variant 1 / 11
    {256, 64, 256, 64},       // 21: d+ <= 64, bucket tables
    {256, 64, 256, 64},       // 22: d+ <= 64, cuckoo tables
    {128, 128, 512, 256},     // 23: d+ <= 256, two wavefronts per node, half-full cuckoo table
    {256, 256, 1024, 512},    // 24: d+ <= 512, four wavefronts per node, half-full cuckoo table
    {512, 512, 1024, 512},    // 25: d+ <= 512, eight wavefronts per node, half-full cuckoo table
    {1024, 1024, 2048, 1024}, // 26: d+ <= 1024, sixteen wavefronts per node, half-full cuckoo table
};
static constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kVariantGlobal = 8;
constexpr int kVariantBitmap = 9;

int count_variant_valid(int v) { return v >= 0 && v < kNumVariants; }
int count_variant_capacity(int v) { return count_variant_valid(v) ? kVariants[v].cap : -1; }
int count_variant_min_side(int v) { return count_variant_valid(v) && kVariants[v].slots > 0; }

template <int NT, int G, int SLOTS, int CAP, bool CK = false, int U = 8>
static void launch_ms(const BinLaunch& b, const int64_t* doff, const int32_t* dcol, unsigned long long* T,
                      unsigned long long* tot, hipStream_t s) {
  constexpr int GPB = NT / G;
  const int64_t nbu = ((int64_t)b.count + GPB - 1) / GPB;
  const int64_t nbw = (b.in_items + GPB - 1) / GPB;
  if (nbu + nbw == 0) return;
  InItems in{b.in_list, b.in_coff, b.in_owner, b.in_base, b.in_nodes, b.in_items};
  k_count_ms<NT, G, SLOTS, CAP, U, CK><<<(unsigned)(nbu + nbw), NT, 0, s>>>(b.list, b.count, in, b.w_max, doff, dcol,
                                                                        b.dinoff, b.dincol, T, tot);
}

template <bool CK, int U = 8>
static void launch_mss(const BinLaunch& b, const int64_t* doff, const int32_t* dcol, unsigned long long* T,
                       unsigned long long* tot, hipStream_t s) {
  constexpr int NT = 256, GS = kSmallGS, GPB = NT / kWave;
  const int64_t nbu = ((int64_t)b.count + GPB * (kWave / GS) - 1) / (GPB * (kWave / GS));
  const int64_t nbw = (b.in_items + GPB - 1) / GPB;
  if (nbu + nbw == 0) return;
  InItems in{b.in_list, b.in_coff, b.in_owner, b.in_base, b.in_nodes, b.in_items};
  k_count_mss<NT, 256, 64, U, CK, GS><<<(unsigned)(nbu + nbw), NT, 0, s>>>(b.list, b.count, in, b.w_max, doff, dcol,
                                                                       b.dinoff, b.dincol, T, tot);
}

// Hub bitmaps: one bit per node id, as many bitmaps as fit 256 MB (8 to 256,
// one per block of the hub variant's grid).
int64_t hub_map_words(int64_t n) { return (n + 31) / 32 > 0 ? (n + 31) / 32 : 1; }
int32_t hub_map_slots(int64_t n) {
  const int64_t fit = (int64_t(256) << 20) / (4 * hub_map_words(n));
  return (int32_t)(fit < 8 ? 8 : fit > 256 ? 256 : fit);
}

hipError_t launch_count_bin(const BinLaunch& b, const int64_t* doff, const int32_t* dcol,
                            unsigned long long* T, unsigned long long* tot, hipStream_t s) {
  if (b.count <= 0 && b.in_items <= 0) return hipSuccess;
  switch (b.variant) {
    case 0: launch_ms<256, 64, 128, 16>(b, doff, dcol, T, tot, s); break;
    case 1: launch_ms<256, 64, 256, 64>(b, doff, dcol, T, tot, s); break;
    case 2: launch_ms<256, 256, 1024, 256>(b, doff, dcol, T, tot, s); break;
    case 3: launch_ms<512, 512, 4096, 1024>(b, doff, dcol, T, tot, s); break;
    case 4: launch_ms<1024, 1024, 8192, 4096>(b, doff, dcol, T, tot, s); break;
    case 5: launch_ms<512, 512, 2048, 1024>(b, doff, dcol, T, tot, s); break;
    case 6: launch_ms<512, 512, 4096, 2048>(b, doff, dcol, T, tot, s); break;
    case 7: launch_ms<256, 256, 512, 256>(b, doff, dcol, T, tot, s); break;
    case 10: launch_ms<256, 64, 128, 16, true>(b, doff, dcol, T, tot, s); break;
    case 11: launch_ms<256, 64, 256, 64, true>(b, doff, dcol, T, tot, s); break;
    case 12: launch_ms<256, 256, 1024, 256, true>(b, doff, dcol, T, tot, s); break;
    case 13: launch_ms<512, 512, 4096, 1024, true>(b, doff, dcol, T, tot, s); break;
    case 14: launch_ms<1024, 1024, 8192, 4096, true>(b, doff, dcol, T, tot, s); break;
    case 15: launch_ms<512, 512, 2048, 1024, true>(b, doff, dcol, T, tot, s); break;
    case 16: launch_ms<512, 512, 4096, 2048, true>(b, doff, dcol, T, tot, s); break;
    case 17: launch_ms<256, 256, 512, 256, true>(b, doff, dcol, T, tot, s); break;
    case 18: launch_ms<128, 128, 512, 128, true>(b, doff, dcol, T, tot, s); break;
    case 19: launch_ms<128, 128, 1024, 256, true>(b, doff, dcol, T, tot, s); break;
    case 20: launch_ms<1024, 1024, 4096, 2048, true>(b, doff, dcol, T, tot, s); break;
    case 21: launch_mss<false>(b, doff, dcol, T, tot, s); break;
    case 22: launch_mss<true>(b, doff, dcol, T, tot, s); break;
    case 23: launch_ms<128, 128, 512, 256, true>(b, doff, dcol, T, tot, s); break;
    case 24: launch_ms<256, 256, 1024, 512, true>(b, doff, dcol, T, tot, s); break;
    case 25: launch_ms<512, 512, 1024, 512, true>(b, doff, dcol, T, tot, s); break;
    case 26: launch_ms<1024, 1024, 2048, 1024, true>(b, doff, dcol, T, tot, s); break;
    case kVariantGlobal:
      k_count_global<<<(unsigned)b.count, 256, 0, s>>>(b.list, b.count, doff, dcol, T, tot);
      break;
    case kVariantBitmap:
      if (!b.hubmap || b.hub_slots < 1) return hipErrorInvalidValue;
      k_count_bitmap<8><<<(unsigned)min(b.count, b.hub_slots), kHubNT, 0, s>>>(b.list, b.count, b.hubmap, b.map_words,
                                                                             doff, dcol, T, tot);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Clears T[n] and the kTotSlots total counters.
__global__ __launch_bounds__(256) void k_zero_counts(unsigned long long* __restrict__ T, int64_t n,
                                                     unsigned long long* __restrict__ tot) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 < kTotSlots) tot[i0] = 0ull;
  for (int64_t i = i0; i < n; i += stride) T[i] = 0ull;
}

hipError_t launch_zero_counts(unsigned long long* T, int64_t n, unsigned long long* tot, hipStream_t s) {
  int64_t g = (std::max<int64_t>(n, kTotSlots) + 255) / 256;
  if (g > 65536) g = 65536;
  k_zero_counts<<<(unsigned)g, 256, 0, s>>>(T, n, tot);
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

// The total from the intersection kernels' counters (not from T), the
// average from the epilogue's FP64 partials in block order, and sum_T =
// sum of the per-node counts (3x the total when both are right).
__global__ __launch_bounds__(256) void k_finish(int64_t nb, int32_t n, const double* __restrict__ part_cc,
                                                const unsigned long long* __restrict__ part_T,
                                                const unsigned long long* __restrict__ tot,
                                                unsigned long long* __restrict__ total, double* __restrict__ avg,
                                                unsigned long long* __restrict__ sum_T) {
  __shared__ double red_d[256 / kWave];
  __shared__ unsigned long long red_t[256 / kWave];
  double acc = 0.0;
  unsigned long long tacc = 0;
  for (int64_t i = threadIdx.x; i < nb; i += 256) { acc += part_cc[i]; tacc += part_T[i]; }
  const double s = block_sum<double, 256>(acc, red_d);
  const unsigned long long st = block_sum<unsigned long long, 256>(tacc, red_t);
  const unsigned long long all = sum_total(tot, red_t);
  if (threadIdx.x == 0) {
    *total = all;
    *avg = n > 0 ? s / (double)n : 0.0;
    *sum_T = st;
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
                         const unsigned long long* tot, unsigned long long* total, double* avg,
                         unsigned long long* sum_T, hipStream_t s) {
  k_finish<<<1, 256, 0, s>>>(nb, n, part_cc, part_T, tot, total, avg, sum_T);
  return hipGetLastError();
}

}  // namespace tricc

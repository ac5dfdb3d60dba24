// Internal launchers of the gfx950 kernels (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tricc {

// ---- CSR build (symmetrise, drop loops, sort rows, dedup) ----------------
// Row length classes used by the segmented row sort.
enum RowClass : int {
  kRowTrivial = 0,  // len <= 1
  kRow8, kRow16, kRow32, kRow64,  // register bitonic sort by a lane group
  kRow128, kRow256, kRow512, kRow1024,  // register bitonic sort by a wavefront
  kRowLds4k,   // <= 4096, register bitonic sort by a block of 4 wavefronts
  kRowLds8k,   // <= 8192, register bitonic sort by a block of 8 wavefronts
  kRowLds32k,  // <= 32768: <= 16384 by a block of 16 wavefronts, longer by an LDS bitonic sort
  kRowLarge,   // > 32768: chunk sort + merge passes
  kNumRowClasses
};
constexpr int kLargeChunk = 32768;

hipError_t launch_degree_raw(const int32_t* src, const int32_t* dst, int64_t m_raw, int32_t n,
                             int32_t* cnt, int32_t* err, hipStream_t s);
// out[0..n] = exclusive prefix sum of in[0..n), out[n] = total.
// `tmp` needs scan_tmp_elems(n) int64 slots.
int64_t scan_tmp_elems(int64_t n);
hipError_t launch_scan_i32(const int32_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s);
hipError_t launch_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s);
hipError_t launch_scatter(const int32_t* src, const int32_t* dst, int64_t m_raw, const int64_t* off,
                          int32_t* cur, int32_t* adj, hipStream_t s);
// Partitioned raw rows (same result as degree_raw + scan + scatter, rows
// unsorted): part_bits(n) is log2 of the nodes per partition, or -1 where
// the partitioned path does not apply (n == 0 or more than kPartMax
// partitions). Staging: pv and pu hold 2 * m_raw entries; ptotal and pcur
// P zeroed counters; pstart and cstart P + 1 slots.
constexpr int kPartMaxParts = 4096;
int part_bits(int64_t n);
hipError_t launch_part_count(const int32_t* src, const int32_t* dst, int64_t m_raw, int32_t n, int pbits, int32_t P,
                             uint32_t* ptotal, int32_t* err, hipStream_t s);
hipError_t launch_part_scan(const uint32_t* ptotal, int32_t P, int64_t* pstart, int64_t* cstart, hipStream_t s);
hipError_t launch_part_place(const int32_t* src, const int32_t* dst, int64_t m_raw, int pbits, int32_t P,
                             const int64_t* pstart, uint32_t* pcur, int32_t* pv, uint16_t* pu, hipStream_t s);
// pass 0: len (zeroed) = raw row lengths; pass 1 (after raw_off = scan of
// len, cur zeroed): adj rows filled.
hipError_t launch_part_rows(int pass, int pbits, int32_t P, int32_t n, int64_t max_entries, const int64_t* pstart,
                            const int64_t* cstart, const uint16_t* pu, const int32_t* pv, int32_t* len,
                            const int64_t* raw_off, int32_t* cur, int32_t* adj, hipStream_t s);
// Classification with per-block histograms (see build_kernels.hip): pass 0
// fills hist[c * nblk + blk]; after an exclusive scan of hist into off,
// pass 1 writes the members of class c at list[off[c * nblk] ...].
int64_t classify_blocks(int64_t n);
// rows by raw length (rows of length <= 1 are not listed; pass 0 sets their deg)
hipError_t launch_classify_rows(int pass, int32_t n, const int32_t* len, int32_t* deg, int32_t* hist,
                                const int64_t* off, int64_t nblk, int32_t* list, hipStream_t s);
// out[i] = prefix[at[i]] for i < k (k <= 64)
hipError_t launch_gather_offsets(const int64_t* prefix, const int64_t* at, int k, int64_t* out, hipStream_t s);
// cls_off[c] = off[c * nblk] for c = 0..nc
hipError_t launch_class_offsets(const int64_t* off, int64_t nblk, int nc, int64_t* cls_off, hipStream_t s);
// Sorts + dedups rows of one class in place; writes deg.
hipError_t launch_sort_rows(int cls, const int32_t* rows, int32_t nrows, const int64_t* off,
                            const int32_t* len, int32_t* adj, int32_t* deg, hipStream_t s);
// Large rows: sort chunks of kLargeChunk in place (no dedup).
hipError_t launch_sort_chunks(const int64_t* chunk_beg, const int32_t* chunk_len, int32_t nchunks,
                              int32_t* buf, hipStream_t s);
// One merge pass: job k merges buf_in[a_beg, a_beg+la) with
// buf_in[a_beg+la, a_beg+la+lb) into buf_out[out_beg, ...). tile_off is the
// prefix of per-job tiles of kMergeTile outputs.
constexpr int kMergeTile = 2048;
hipError_t launch_merge_pass(const int64_t* a_beg, const int32_t* la, const int32_t* lb,
                             const int64_t* out_beg, const int64_t* tile_off, int32_t njobs,
                             int64_t ntiles, const int32_t* buf_in, int32_t* buf_out, hipStream_t s);
// Dedups sorted large rows from `sorted` (segment seg_beg[i]) into adj at
// off[row[i]], writes deg.
hipError_t launch_dedup_rows(const int32_t* rows, const int64_t* seg_beg, int32_t nrows,
                             const int32_t* len, const int32_t* sorted, const int64_t* off,
                             int32_t* adj, int32_t* deg, hipStream_t s);

// ---- Degree-order orientation --------------------------------------------
// One pass over every row: dplus[v] = |{w in N(v): (d(v),v) < (d(w),w)}|,
// stats[0] = max d, stats[1] = max d+, and row v partitioned into
// part[off[v] .. off[v] + d(v)): N+(v) ascending from the front, N-(v) from
// the back in reverse. Rows of raw length > 64 must be listed: medium_rows
// (a wavefront each) and long_rows (a block each) together. cls: scratch of
// ceil(n / 16) words for the key classes of the rank test. key (may be
// null: the degrees) replaces d in the rank (key(v), v); it must hold
// non-negative values.
hipError_t launch_orient(int32_t n, const int64_t* off, const int32_t* len, const int32_t* deg, const int32_t* key,
                         const int32_t* adj, const int32_t* medium_rows, int32_t nmedium, const int32_t* long_rows,
                         int32_t nlong, uint32_t* cls, int32_t* dplus, int32_t* part, int32_t* stats, hipStream_t s);
// After doff / dinoff are the scans of d+ / d-: N+(v) to dcol[doff[v]..] and
// (dincol != NULL) N-(v) to dincol[dinoff[v]..], both ascending.
hipError_t launch_orient_copy(int32_t n, const int64_t* off, const int32_t* len, const int32_t* deg,
                              const int32_t* dplus, const int32_t* part, const int32_t* medium_rows, int32_t nmedium,
                              const int32_t* long_rows, int32_t nlong, const int64_t* doff, int32_t* dcol,
                              const int64_t* dinoff, int32_t* dincol, hipStream_t s);

// din = deg - dplus; *deg2 (zeroed) += nodes with deg >= 2
hipError_t launch_indeg(int32_t n, const int32_t* deg, const int32_t* dplus, int32_t* din, int32_t* deg2,
                        hipStream_t s);
// Caller CSR: bounds check (err bit 4; sets len and deg when non-null), row
// check (bit 1: id out of range, bit 2: not strictly ascending or a self
// loop; only after the bounds check passed), expansion into (v, w) pairs.
hipError_t launch_csr_bounds(int32_t n, int64_t nnz, const int64_t* rowptr, int32_t* len, int32_t* deg, int32_t* err,
                             hipStream_t s);
hipError_t launch_csr_rows(int32_t n, const int64_t* rowptr, const int32_t* col, int32_t* err, hipStream_t s);
hipError_t launch_csr_expand(int32_t n, const int64_t* rowptr, int32_t* src, hipStream_t s);
// in-list pass owners by d+(w) into bins 0..kNumBins-2 (see InBinOf)
hipError_t launch_classify_inbins(int pass, int32_t n, const int32_t* dplus, const int32_t* deg, const int32_t* limit,
                                  int32_t* hist, const int64_t* off, int64_t nblk, int32_t* list, hipStream_t s);
// nch[i] = ceil(d-(list[i]) / cap_of[bin of i])
hipError_t launch_in_chunks(const int32_t* list, int64_t nlist, const int32_t* din, const int32_t* cap_of,
                            const int64_t* bin_off, int32_t* nch, hipStream_t s);
// owner[c] = i for each in-list chunk c in [coff[i], coff[i+1]), i < nlist
hipError_t launch_in_owners(int64_t nlist, const int64_t* coff, int32_t* owner, hipStream_t s);

hipError_t launch_list_elems(int32_t n, const int64_t* doff, const int32_t* dcol, unsigned long long* out,
                             hipStream_t s);
hipError_t launch_gather_rows(const int32_t* rows, int32_t nr, const int64_t* off, const int32_t* len,
                              int64_t* out_off, int32_t* out_len, hipStream_t s);

// ---- Work binning for the intersection kernels ---------------------------
constexpr int kNumBins = 6;
// Node u with d+(u) >= 2 goes to the first bin b with d+(u) <= limit[b];
// bin kNumBins-1 takes the rest.
hipError_t launch_classify_bins(int pass, int32_t n, const int32_t* dplus, const int32_t* limit, int32_t* hist,
                                const int64_t* off, int64_t nblk, int32_t* list, hipStream_t s);
// per-bin sums of d+(u) + d+(w), of edges over the DAG edges each bin's
// kernel counts (min-side ownership with w_max; w_max = 0 disables it), and
// of the bytes the min-side kernel moves (din / cap: in-degrees and in-list
// chunk sizes; din may be null when w_max = 0)
hipError_t launch_bin_elems(int32_t n, const int64_t* doff, const int32_t* dcol, const int32_t* din,
                            const int32_t* limit, const int32_t* cap, int32_t w_max, unsigned long long* elems,
                            unsigned long long* edges, unsigned long long* kbytes, hipStream_t s);
hipError_t launch_probe_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// ---- Intersection and epilogue --------------------------------------------
struct BinLaunch {
  int variant;  // kernel variant id (see count_kernels.hip)
  const int32_t* list;
  int32_t count;
  // min-side variants only: the bin's in-list items and the ownership bound
  const int32_t* in_list = nullptr;
  const int64_t* in_coff = nullptr;
  const int32_t* in_owner = nullptr;  // owner index (+ in_base) of each of the bin's chunks
  int32_t in_base = 0;
  int32_t in_nodes = 0;
  int64_t in_items = 0;
  int32_t w_max = 0;
  const int64_t* dinoff = nullptr;
  const int32_t* dincol = nullptr;
  // hub bitmap variant only: hub_slots zeroed bitmaps of map_words words
  uint32_t* hubmap = nullptr;
  int32_t hub_slots = 0;
  int64_t map_words = 0;
};
// Bitmaps for the hub variant: words per bitmap and how many fit the region.
int64_t hub_map_words(int64_t n);
int32_t hub_map_slots(int64_t n);
// Counters of the triangle total, fed by the intersection kernels apart from
// T (each node group adds the triangles it found to counter blockIdx % this).
constexpr int kTotSlots = 512;
hipError_t launch_count_bin(const BinLaunch& b, const int64_t* doff, const int32_t* dcol,
                            unsigned long long* T, unsigned long long* tot, hipStream_t s);
int count_variant_capacity(int variant);  // max d+(u) a variant accepts
int count_variant_valid(int variant);
int count_variant_min_side(int variant);  // out-list + in-list kernel
// Clears T[n] and tot[kTotSlots].
hipError_t launch_zero_counts(unsigned long long* T, int64_t n, unsigned long long* tot, hipStream_t s);
// cc[v] (fp32) from T and deg; block partials of the FP64 ratio sum and of T.
int64_t epilogue_blocks(int64_t n);
hipError_t launch_epilogue(int32_t n, const unsigned long long* T, const int32_t* deg, float* cc,
                           double* part_cc, unsigned long long* part_T, hipStream_t s);
// *total = sum of tot (the intersection kernels' own count), *avg from the
// FP64 partials, *sum_T = sum of the T partials.
hipError_t launch_finish(int64_t nb, int32_t n, const double* part_cc, const unsigned long long* part_T,
                         const unsigned long long* tot, unsigned long long* total, double* avg,
                         unsigned long long* sum_T, hipStream_t s);

// ---- Batched graphs ---------------------------------------------------------
// Persistent intersection kernel over four node lists (hubs -> global
// fallback, block nodes, single-wave nodes, short-list nodes); queue[0] and
// the queue counters must be 0 at launch (launch_batch_zero clears them).
int persist_variant_count();
int persist_wave_cap(int v);   // largest d+ of a single-wave node
int persist_block_cap(int v);  // largest d+ of a block node
int persist_merge_cap(int v);  // largest merge_limit the variant accepts
const void* persist_kernel(int v);
// Phase 2 of the persistent kernel runs in kPersistSegs segments (one per
// XCD of the chip: 256 CUs in 8 XCDs); seg holds 2 (kPersistSegs + 1) bounds
// (launch_persist_segments); queue needs 2 + kPersistSegs counters.
constexpr int kPersistSegs = 8;
hipError_t launch_count_persist(int v, unsigned grid, const int32_t* glist, int32_t ng, const int32_t* blist,
                                int32_t nbk, const int32_t* wlist, const int32_t* mlist, const int32_t* seg,
                                int32_t* queue, const int64_t* doff, const int32_t* dcol, unsigned long long* T,
                                unsigned long long* tot, hipStream_t s);
// Bounds of the segments in wlist[0, nw) and mlist[0, nm): thr[x] (x = 0 ..
// kPersistSegs) is the first node id of segment x.
hipError_t launch_persist_segments(const int32_t* wlist, int32_t nw, const int32_t* mlist, int32_t nm,
                                   const int64_t* thr, int32_t* out, hipStream_t s);
hipError_t launch_batch_zero(unsigned long long* T, int64_t n, unsigned long long* tot, int32_t* queue,
                             hipStream_t s);
// batch_tri (may be null): the batch's total from tot.
hipError_t launch_graph_epilogue(int32_t num_graphs, const int64_t* node_off, const unsigned long long* T,
                                 const int32_t* deg, float* cc, unsigned long long* graph_tri, double* graph_avg,
                                 const unsigned long long* tot, unsigned long long* batch_tri, hipStream_t s);
// Local -> global ids of a packed batch: edge e of graph g gets node_off[g]
// added; err is set if a local id is outside [0, n_g).
hipError_t launch_batch_relabel(int32_t num_graphs, const int64_t* node_off, const int64_t* edge_off,
                                const int32_t* src, const int32_t* dst, int64_t m_raw, int32_t* gsrc,
                                int32_t* gdst, int32_t* err, hipStream_t s);

// ---- Edge-existence tests ---------------------------------------------------
// Records of the simple graph whose row v is adj[off[v] .. off[v] + deg[v])
// ascending: rec[2v] = off[v] as uint32 (offsets stay below 2^32), rec[2v+1]
// = deg[v]; 8-byte aligned, 2n int32.
hipError_t launch_edge_records(int32_t n, const int64_t* off, const int32_t* deg, int32_t* rec, hipStream_t s);
// out[i] = 1 if {qu[i], qv[i]} is an edge, 0 if not (qu[i] == qv[i]
// included), kEdgeQueryBadId if an id lies outside [0, n).
constexpr uint8_t kEdgeQueryBadId = 0xFF;
hipError_t launch_has_edges(int64_t q, const int32_t* qu, const int32_t* qv, int32_t n, const int32_t* rec,
                            const int32_t* adj, uint8_t* out, hipStream_t s);

// ---- Core numbers ------------------------------------------------------------
// Level-synchronous peeling over the simple graph's rows (row v =
// adj[off[v] .. off[v] + deg[v])). cur, F, G, A, S, and the two near lists:
// int32[n] scratch; core: int32[n] (-1 while a node is left); cnt: int32[8]
// counters (see core_kernels.hip). The scan visits the listed candidates
// A[0, na) (A == NULL: all ids), lists the other nodes left in S (if not
// NULL) and those of them with current degree <= U in the near list Nr (if
// not NULL; its length in *ncnt).
hipError_t launch_core_init(int32_t n, const int32_t* deg, int32_t* cur, int32_t* core, hipStream_t s);
// which 0: frontier, minimum and survivor counters; 1: next-frontier
// counter; near >= 0: also clears cnt[near]
hipError_t launch_core_reset(int32_t* cnt, int which, int near, hipStream_t s);
// order (may be null): removal round of each node taken, `round` for the
// scan's frontier and round + 1 for the peel's next frontier.
hipError_t launch_core_scan(int32_t na, const int32_t* A, int32_t k, const int32_t* cur, int32_t* core, int32_t* F,
                            int32_t* S, int32_t* cnt, int32_t* order, int32_t round, int32_t U, int32_t* Nr,
                            int32_t* ncnt, hipStream_t s);
// Nr (may be null): a node whose current degree falls from U + 1 to U is
// appended to it (*ncnt its length).
hipError_t launch_core_peel(const int32_t* F, int32_t nf, int32_t k, const int64_t* off, const int32_t* deg,
                            const int32_t* adj, int32_t* cur, int32_t* core, int32_t* G, int32_t* cnt, int32_t* order,
                            int32_t round, int32_t U, int32_t* Nr, int32_t* ncnt, hipStream_t s);
// core_peel_batch() rounds of one level: the frontier starts in B0 (nf
// nodes) and alternates between B0 and B1; round i counts its next frontier
// in cnt[16 + i] (cleared here) and takes the order value round + i + 1 for
// it. Round i > 0 reads its size from cnt[16 + i - 1]; an empty round does
// nothing. With an even batch the frontier left ends in B0.
int core_peel_batch();
hipError_t launch_core_peel_batch(int32_t* B0, int32_t* B1, int32_t nf, int32_t k, const int64_t* off,
                                  const int32_t* deg, const int32_t* adj, int32_t* cur, int32_t* core, int32_t* cnt,
                                  int32_t* order, int32_t round, int32_t U, int32_t* Nr, int32_t* ncnt,
                                  hipStream_t s);
hipError_t launch_core_fill(int32_t n, int32_t k, int32_t* core, hipStream_t s);

// ---- 4-clique counts ---------------------------------------------------------
// *total = number of 4-cliques, over the DAG N+(v) = dcol[doff[v] ..
// doff[v+1]) (ascending ids); every d+(v) must be <= kK4Cap (bit rows over
// blocks of positions index at most this many).
constexpr int32_t kK4Cap = 8192;
hipError_t launch_count_k4(int32_t n, const int64_t* doff, const int32_t* dcol, unsigned long long* total,
                           hipStream_t s);
// *total = number of 5-cliques over the same DAG; every d+(v) must be <=
// kK5Cap (the bit rows of one node, whole, in LDS).
constexpr int32_t kK5Cap = 1024;
hipError_t launch_count_k5(int32_t n, const int64_t* doff, const int32_t* dcol, unsigned long long* total,
                           hipStream_t s);

// R-MAT edges 0..m-1 with 2^scale nodes (a, b, c, d quadrant weights, noise
// in [0, 1]), counter-based from seed; perm (2^scale ids, may be null)
// relabels both ends.
hipError_t launch_gen_rmat(int64_t m, int scale, const double abcd[4], double noise, uint64_t seed,
                           const int32_t* perm, int32_t* src, int32_t* dst, hipStream_t s);

// Erdos-Renyi G(n, m) as the first m distinct draws of a counter-based
// sequence over the N = n(n-1)/2 pair indices (seed stream 13): keys/idx a
// table of P (a power of two, >= 2K) slots, cleared first; K draws inserted;
// flag[k] = draw k is the first of its value; pos = exclusive scan of flag;
// emit writes the new draws with pos[k] < m as edges pos[k].
hipError_t launch_er_clear(uint64_t P, uint64_t* keys, uint32_t* idx, hipStream_t s);
hipError_t launch_er_insert(int64_t K, uint64_t N, uint64_t seed, uint64_t mask, uint64_t* keys, uint32_t* idx,
                            hipStream_t s);
hipError_t launch_er_flag(int64_t K, uint64_t N, uint64_t seed, uint64_t mask, const uint64_t* keys,
                          const uint32_t* idx, int32_t* flag, hipStream_t s);
hipError_t launch_er_emit(int64_t K, int64_t n, uint64_t N, uint64_t seed, int64_t m, const int32_t* flag,
                          const int64_t* pos, int32_t* src, int32_t* dst, hipStream_t s);
// Barabasi-Albert with k distinct targets per node (seed stream 14): init
// writes the seed clique and every source, clears prog[n] and cnt[2]; each
// pass resolves what it can, cnt[0] = nodes left, cnt[1] = attempts ran out.
hipError_t launch_ba_init(int64_t m, int32_t k, int32_t n, int32_t* src, int32_t* dst, int32_t* prog, int32_t* cnt,
                          hipStream_t s);
hipError_t launch_ba_pass(int32_t n, int32_t k, uint64_t seed, const int32_t* src, int32_t* dst, int32_t* prog,
                          int32_t* cnt, hipStream_t s);

}  // namespace tricc

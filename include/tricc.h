/*
 * tricc — exact triangle counting and clustering coefficients on MI355X
 * (gfx950), C ABI.
 *
 * The operation (paper: SNAP, Leskovec and Sosic, ACM TIST 2016; Section 4,
 * table of graph analytics methods, "triadic closure": node clustering
 * coefficient and triangle counting). The paper names the methods without
 * formulas; this library computes the plain definitions:
 *
 *   E     = { {u,v} : (u,v) or (v,u) in the input edge list, u != v }
 *           (undirected simple graph: Section 3.1 — undirected graphs, edges
 *           as node pairs without ids; duplicates and self loops are dropped)
 *   N(v)  = neighbours of v, d(v) = |N(v)|  (Section 5.1: a sorted vector of
 *           adjacent nodes per node)
 *   T(v)  = number of triangles that contain v
 *   T     = number of triangles (each counted once; sum_v T(v) = 3 T)
 *   CC(v) = 2 T(v) / (d(v) (d(v) - 1)) if d(v) >= 2, else 0   (FP32)
 *   avg   = (1/n) sum over all n node ids of CC(v)             (FP64)
 *
 * Nodes are the dense ids 0..n-1 (Section 3.1 allows any non-negative id;
 * relabel to a dense range first). Isolated ids are nodes with CC 0 and
 * count in the average.
 *
 * Conventions for every call:
 *   - Pointers named d_* are device pointers (HIP device memory, e.g. the
 *     data of a torch CUDA tensor); h_* are host pointers.
 *   - The caller owns every buffer it passes and must keep the workspace
 *     alive while a handle built on it is in use. Handles are owned by the
 *     library and released with the matching *_free call.
 *   - `stream` is a hipStream_t (NULL = the null stream). Calls documented
 *     as asynchronous only enqueue work on it.
 *   - Return value: a TRICC_* status. No C++ exception crosses the ABI. The
 *     text of the last error of the calling thread is tricc_last_error().
 *   - Node ids are int32 in [0, n), n < 2^31 - 1. Counts are uint64.
 */
#ifndef TRICC_H_
#define TRICC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRICC_OK 0
#define TRICC_EINVAL 1    /* bad argument */
#define TRICC_ERANGE 2    /* a node id outside [0, n) */
#define TRICC_ENOMEM 3    /* workspace or memory budget too small */
#define TRICC_EHIP 4      /* HIP runtime error, see tricc_last_error() */
#define TRICC_EBUSY 5     /* admission refused: retry later */
#define TRICC_EOVERFLOW 6 /* a size exceeds what the library supports */

#define TRICC_NUM_BINS 6

/* Degree-binned scheduling of the intersection kernels. A node u with
 * out-degree d+(u) >= 2 in the degree-ordered DAG goes to the first bin b
 * with d+(u) <= bin_limit[b] (bins 0..4), else to bin 5; bin b runs the
 * kernel variant bin_variant[b]. A variant's capacity (the largest d+ it
 * accepts, tricc_variant_capacity) must cover the largest d+ of its bin.
 *
 * min_side = 1: every DAG edge u->w is counted by streaming the shorter of
 * the two out-lists: edges with d+(u) < d+(w) <= bin_limit[4] are counted
 * from w (its out-list is the LDS table, u's out-list is streamed). This
 * needs the min-side kernel variants (tricc_variant_min_side) in bins 0..4;
 * with min_side = 0 those variants count every edge from its tail. */
typedef struct tricc_tuning {
  int32_t bin_limit[TRICC_NUM_BINS - 1];
  int32_t bin_variant[TRICC_NUM_BINS];
  int32_t min_side;
} tricc_tuning;

typedef struct tricc_graph_info {
  int32_t n;
  int64_t m_raw;               /* input pairs */
  int64_t m;                   /* undirected simple edges (= DAG edges) */
  int64_t max_deg;             /* max d(v) */
  int64_t max_outdeg;          /* max d+(v) */
  int64_t bin_count[TRICC_NUM_BINS];
  uint64_t list_elems;         /* sum over DAG edges u->w of d+(u) + d+(w) (*) */
  int64_t large_rows;          /* rows sorted by the chunk + merge path */
  uint64_t bin_list_elems[TRICC_NUM_BINS]; /* d+(u) + d+(w) over the edges each bin's kernel counts (*) */
  int64_t bin_edges[TRICC_NUM_BINS];       /* DAG edges counted by each bin's kernel (*) */
  int64_t bin_in_items[TRICC_NUM_BINS];    /* in-list work items of each bin (min-side) */
  int64_t n_deg2;              /* nodes with d(v) >= 2; the average CC over these nodes alone is
                                  avg * n / n_deg2 (every other node has CC 0) */
  uint64_t bin_kernel_bytes[TRICC_NUM_BINS]; /* bytes each bin's min-side kernel reads and writes when
                                  nothing is reused between its work items: out-list tables, row
                                  bounds, streamed (shorter) lists, in-list chunks, credits (*) */
  /* (*) zero until tricc_graph_stats has run */
} tricc_graph_info;

typedef struct tricc_graph tricc_graph;

const char* tricc_status_str(int status);
/* Last error text of the calling thread ("" if none). */
const char* tricc_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int tricc_version(void);

/* Default tuning (no device access). */
int tricc_default_tuning(tricc_tuning* out);
/* Largest d+ a kernel variant accepts; -1 if the variant does not exist. */
int tricc_variant_capacity(int variant);
/* Number of kernel variants (valid ids are 0 .. count-1):
 *   0..7    LDS bucket tables (capacities 16, 64, 256, 1024, 4096, 1024,
 *           2048, 256), one node per group of 64..1024 lanes
 *   8       N+(u) binary-searched in HBM (any d+)
 *   9       N+(u) as a bitmap over all ids in HBM (any d+; the default for
 *           nodes above every LDS table)
 *   10..17  as 0..7 with two-choice cuckoo tables
 *   18, 19  cuckoo tables for d+ <= 128 and <= 256, two wavefronts per node
 *   20      cuckoo table of 4,096 slots for d+ <= 2048, sixteen wavefronts
 *           per node (two blocks fill a CU's wave slots)
 *   21, 22  d+ <= 64: four nodes with d+ <= 16 per wavefront (one 64-slot
 *           table each), the bin's other nodes one per wavefront as 1 / 11;
 *           21 bucket tables, 22 cuckoo tables
 *   23..26  cuckoo tables up to half full: 512 slots for d+ <= 256 (two
 *           wavefronts per node), 1,024 slots for d+ <= 512 (four or eight
 *           wavefronts), 2,048 slots for d+ <= 1024 (sixteen wavefronts) */
int tricc_variant_count(void);
/* 1 if the variant implements both sides of the min-side split (every
 * variant but 8 and 9). */
int tricc_variant_min_side(int variant);

/* Bytes of device workspace tricc_graph_build needs for (n, m_raw). */
int tricc_graph_workspace_size(int32_t n, int64_t m_raw, size_t* bytes);

/*
 * Steps a1..a5 of the path: validate, symmetrise, drop self loops, sort each
 * row and drop duplicates (CSR of the simple graph), orient every edge from
 * the lower to the higher (degree, id) rank (a DAG whose out-degrees are at
 * most sqrt(2m)), and bin the DAG's nodes for the intersection kernels.
 *   n        number of nodes (0 <= n < 2^31 - 1)
 *   m_raw    number of input pairs (0 <= m_raw <= 2^30)
 *   d_src, d_dst  device int32[m_raw]: pair e is (d_src[e], d_dst[e]);
 *                 any order, duplicates and self loops allowed
 *   d_ws, ws_bytes  device workspace of at least tricc_graph_workspace_size
 *   tuning   NULL for the default
 * Synchronises `stream` (sizes of later launches are read back).
 * Errors: TRICC_ERANGE if any id is outside [0, n) (no handle is made),
 * TRICC_ENOMEM if ws_bytes is too small, TRICC_EINVAL on bad sizes or tuning.
 */
int tricc_graph_build(int32_t n, int64_t m_raw, const int32_t* d_src, const int32_t* d_dst,
                      void* d_ws, size_t ws_bytes, const tricc_tuning* tuning, void* stream,
                      tricc_graph** out);

/*
 * Steps a1..a5 from a graph the caller holds as a CSR: row v is
 * d_col[d_rowptr[v] .. d_rowptr[v+1]) (the paper's per-node sorted
 * neighbour vectors, Section 5.1, laid end to end).
 *   n, nnz      nodes and entries (d_rowptr[n] must equal nnz <= 2^30)
 *   d_rowptr    device int64[n+1], from 0, non-decreasing; d_col device int32[nnz]
 *   assume_simple_sorted_symmetric
 *     0: each entry w of row v is taken as the pair (v, w) and goes through
 *        the full build (symmetrise, dedup, self loops dropped), exactly as
 *        tricc_graph_build on those pairs.
 *     1: the caller asserts that every row is strictly ascending, holds no
 *        self loop, and that w is in row v iff v is in row w; the rows are
 *        copied and the sort is skipped. Ranges, order and loops are checked;
 *        symmetry is not (an asymmetric CSR gives undefined counts, never an
 *        access outside the workspace).
 *   d_ws, ws_bytes  at least tricc_graph_workspace_size(n, nnz); the caller's
 *                   arrays are only read
 * Synchronises `stream`. Errors: TRICC_EINVAL for malformed row offsets, a
 * row that is not strictly ascending or holds its own id (mode 1), bad sizes
 * or tuning; TRICC_ERANGE for an id outside [0, n); TRICC_ENOMEM for a short
 * workspace. No handle is made on error.
 */
int tricc_graph_from_csr(int32_t n, int64_t nnz, const int64_t* d_rowptr, const int32_t* d_col,
                         int assume_simple_sorted_symmetric, void* d_ws, size_t ws_bytes,
                         const tricc_tuning* tuning, void* stream, tricc_graph** out);

int tricc_graph_info_get(const tricc_graph* g, tricc_graph_info* out);

/* Fills the fields of tricc_graph_info marked (*): the algorithmic sizes of
 * the intersection work, from which its algorithmic bytes follow. Not part
 * of the counting path. Synchronises `stream`. */
int tricc_graph_stats(tricc_graph* g, void* stream);

/* Re-bins the graph's nodes with another tuning (clears the (*) fields).
 * Synchronises `stream`. */
int tricc_graph_retune(tricc_graph* g, const tricc_tuning* tuning, void* stream);

/*
 * Steps a6..a7: per-node triangle counts, clustering coefficients, the total
 * and the average. Asynchronous on `stream`.
 *   d_node_tri  device uint64[n] (overwritten)
 *   d_node_cc   device float[n]
 *   d_total     device uint64[1]: the number of triangles as the
 *               intersection kernels found them (each triangle is found by
 *               one node group, which adds it to the total), accumulated
 *               apart from d_node_tri; sum_v T(v) = 3 * total holds when
 *               both are right (tricc_count_check)
 *   d_avg_cc    device double[1]; the FP64 sum is taken in a fixed order,
 *               so repeated calls give bit-identical results.
 * Counts of one graph must not overlap in time (they share the graph's
 * workspace counters and hub bitmaps).
 */
int tricc_count(tricc_graph* g, uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_total,
                double* d_avg_cc, void* stream);

/*
 * The three parts of tricc_count, for callers that time or overlap them:
 * begin zeroes d_node_tri; bin b (0 <= b < TRICC_NUM_BINS) runs the
 * intersection kernel of one bin (no-op for an empty bin); finish runs the
 * epilogue (CC, total, average). Issued in that order on one stream they
 * equal tricc_count. Asynchronous.
 */
int tricc_count_begin(tricc_graph* g, uint64_t* d_node_tri, void* stream);
int tricc_count_bin(tricc_graph* g, int bin, uint64_t* d_node_tri, void* stream);
/*
 * Bins first..last (0 <= first <= last < TRICC_NUM_BINS), which must share
 * one kernel variant in g's tuning, as ONE launch over their contiguous
 * node lists and in-list chunks: what tricc_count issues for each run of
 * adjacent bins with equal variants. TRICC_EINVAL for a bad range or mixed
 * variants (nothing launched). Asynchronous; no-op if the bins are empty.
 */
int tricc_count_bins(tricc_graph* g, int first, int last, uint64_t* d_node_tri, void* stream);
int tricc_count_finish(tricc_graph* g, const uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_total,
                       double* d_avg_cc, void* stream);

/* After a count of g: its total and the sum of its per-node counts, as the
 * device computed them (the sum is taken by the epilogue, the total by the
 * intersection kernels). Synchronises `stream`. */
int tricc_count_check(const tricc_graph* g, uint64_t* h_total, uint64_t* h_sum_T, void* stream);

/* Streaming copy of `bytes` (a multiple of 16, both pointers 16-byte
 * aligned) from d_src to d_dst: the reference kernel for achievable HBM
 * bandwidth and for calibrating memory-traffic counters. Asynchronous. */
int tricc_probe_copy(void* d_dst, const void* d_src, size_t bytes, void* stream);

/*
 * R-MAT edge generator on the device (the paper's table of graph
 * generators, Section 4; R-MAT of Chakrabarti, Zhan and Faloutsos, SDM
 * 2004). Edge e (0 <= e < m) of a graph with n = 2^scale ids is `scale`
 * quadrant choices, most significant bit first. At level l, with
 * k = 2 (e * scale + l) and word(c) = SplitMix64 output of
 * S + c * 0x9E3779B97F4A7C15, S = SplitMix64 output of
 * seed + 12 * 0x9E3779B97F4A7C15:
 *   p_q = w_q * (1 + noise * (2 h_q / 65535 - 1)), h_q = bits 16q..16q+15
 *         of word(k + 1), (w_0..w_3) = (a, b, c, d)            (FP64)
 *   x   = (word(k + 2) >> 11) * 2^-53 * (p_0 + p_1 + p_2 + p_3)
 *   q   = first q with x < p_0 + .. + p_q (else 3); src bit q >> 1, dst bit q & 1
 * every FP64 operation separately rounded, sums left to right, so the
 * edges are exact bit patterns, independent of the launch. Self loops and
 * duplicate pairs are kept (the graph build removes them).
 *   d_perm   device int32[n] (may be NULL): relabelling, both ends
 *            id -> d_perm[id]; must hold ids in [0, n) (not checked)
 *   d_src, d_dst  device int32[m], the caller's (written)
 * Asynchronous on `stream`. Errors: TRICC_EINVAL for scale outside [1, 30],
 * m < 0, weights negative, not finite or summing to 0, noise outside
 * [0, 1], null outputs with m > 0.
 */
int tricc_gen_rmat(int32_t scale, int64_t m, double a, double b, double c, double d, double noise, uint64_t seed,
                   const int32_t* d_perm, int32_t* d_src, int32_t* d_dst, void* stream);

/*
 * Erdos-Renyi G(n, m) on the device (the paper's table of graph generators,
 * Section 4): a uniform random m-subset of the N = n(n-1)/2 node pairs. The
 * definition, written out so that the edges are exact: with word(c) =
 * SplitMix64 output of S + c * 0x9E3779B97F4A7C15 and S = SplitMix64 output
 * of seed + 13 * 0x9E3779B97F4A7C15, draw k (k = 0, 1, ...) is the pair
 * index x_k = floor(word(k + 1) * N / 2^64); the edges are the first m
 * distinct values of x_0, x_1, ... in draw order (edge e = the e-th new
 * value); pair index t is the pair (i, j), i < j, with t = i n - i(i+1)/2 +
 * (j - i - 1), written (i, j), or (j, i) when bit 0 of its word is 1. No
 * self loops, no repeated pair.
 *   n        0 <= n < 2^31; m: 0 <= m <= min(N, 2^30)
 *   d_src, d_dst  device int32[m], the caller's (written)
 *   d_ws     device scratch of tricc_gen_er_workspace_size(n, m) bytes
 *            (256-byte aligned; about 12 bytes per draw slot of a hash table
 *            of at least twice the draws, plus 12 bytes per draw)
 * Synchronises `stream` (the number of distinct draws is read back).
 * Errors: TRICC_EINVAL for n or m out of range, null arrays or a misaligned
 * workspace; TRICC_ENOMEM for a short workspace; TRICC_EOVERFLOW when m is
 * so close to N that the draw budget would pass 2^32 (or, with a chance far
 * below any practical concern, the draws run short of m distinct values).
 */
int tricc_gen_er_workspace_size(int64_t n, int64_t m, size_t* bytes);
int tricc_gen_er(int64_t n, int64_t m, uint64_t seed, int32_t* d_src, int32_t* d_dst, void* d_ws, size_t ws_bytes,
                 void* stream);

/*
 * Barabasi-Albert preferential attachment on the device (the paper's table of
 * graph generators, Section 4), with k distinct targets per node. Definition:
 * nodes 0..k form the clique K_{k+1}, whose edges e = 0 .. k(k+1)/2 - 1 are
 * its pairs (i, j), i < j, in lexicographic order (source i, target j). Node
 * v > k adds edges e = E_v + j, j = 0..k-1, E_v = k(k+1)/2 + (v - k - 1) k,
 * with source v. Edge e' holds its source at endpoint position 2e' and its
 * target at 2e' + 1; the target of edge e = E_v + j is the node at position
 * r = floor(word((e << 20) + a + 1) * 2 E_v / 2^64) (word as for G(n, m),
 * S = SplitMix64 output of seed + 14 * 0x9E3779B97F4A7C15) for the first
 * attempt a = 0, 1, ... whose node is not already a target of v's edges
 * j' < j. Every position holds one endpoint, so a node is drawn in
 * proportion to its degree among the edges before v's. The device resolves
 * the edges in passes: an edge whose draws reach only final targets becomes
 * final; the earliest open edge always can, so every pass makes progress.
 *   m = tricc_gen_ba_edges(n, k) = k(k+1)/2 + (n - k - 1) k  (-1 unless
 *       1 <= k <= 255 and k < n < 2^31); m <= 2^30
 *   d_src, d_dst  device int32[m], the caller's (written)
 *   d_ws     device scratch of tricc_gen_ba_workspace_size(n, k) bytes
 * Synchronises `stream` (the passes read back how many nodes are open).
 * Errors: TRICC_EINVAL for bad sizes or null arrays, TRICC_ENOMEM for a
 * short workspace, TRICC_EOVERFLOW above 2^30 edges (or if an edge needs
 * 2^20 attempts).
 */
int64_t tricc_gen_ba_edges(int64_t n, int32_t k);
int tricc_gen_ba_workspace_size(int64_t n, int32_t k, size_t* bytes);
int tricc_gen_ba(int64_t n, int32_t k, uint64_t seed, int32_t* d_src, int32_t* d_dst, void* d_ws, size_t ws_bytes,
                 void* stream);

/* Device views of the graph held in the workspace, for inspection:
 * row v of the simple graph is d_adj[d_off[v] .. d_off[v] + d_deg[v]) in
 * ascending id order; the DAG out-list of v is d_dcol[d_doff[v] ..
 * d_doff[v+1]) in ascending id order. Any pointer may be NULL. */
int tricc_graph_arrays(const tricc_graph* g, const int64_t** d_off, const int32_t** d_deg,
                       const int32_t** d_adj, const int64_t** d_doff, const int32_t** d_dcol);

/*
 * Edge-existence tests on a built graph (IsEdge, among the graph methods of
 * the paper's Section 4; Section 5.1 tests an edge by searching a node's
 * sorted neighbour vector, O(log deg_max), and Section 6.2 times random
 * tests). Query i asks whether {d_u[i], d_v[i]} is an edge of the simple
 * graph (symmetrised, loops and duplicates dropped); the search runs in
 * the shorter of the two sorted rows, one query per GPU thread.
 *   q           number of queries (>= 0)
 *   d_u, d_v    device int32[q], the caller's; only read
 *   d_out       device uint8[q], the caller's: 1 = edge, 0 = no edge (a pair
 *               (v, v) is never an edge), 0xFF = an id outside [0, n)
 * Asynchronous on `stream`. Reads the graph's rows only, so it may overlap
 * counts of the same graph. Errors: TRICC_EINVAL for a null handle, q < 0,
 * or a null array with q > 0; TRICC_EHIP on a launch failure. An invalid id
 * is reported per query, not as an error.
 */
int tricc_graph_has_edges(const tricc_graph* g, int64_t q, const int32_t* d_u, const int32_t* d_v,
                          uint8_t* d_out, void* stream);

/*
 * Core numbers (k-core analysis, among the analytics methods of the paper's
 * Section 4; Section 5 names the Batagelj-Zaversnik decomposition, and
 * Section 6.3 times the extraction of a 3-core). The k-core is the largest
 * subgraph whose nodes all have degree >= k; the core number of v is the
 * largest k whose k-core holds v. Computed on the GPU by level-synchronous
 * peeling of the simple graph.
 *   k_stop      < 0: every node's core number; >= 0: min(core number,
 *               k_stop), so the k_stop-core is { v : d_core[v] == k_stop }
 *               and the peeling stops at that level
 *   d_core      device int32[n], the caller's (written)
 *   d_ws        device scratch of tricc_core_workspace_size(n) bytes, the
 *               caller's; contents on entry do not matter
 *   h_max_core  host int32 (may be NULL): the largest value written
 * Synchronises `stream` (the peeling loop reads the frontier sizes back).
 * Errors: TRICC_EINVAL for a null handle or null arrays with n > 0,
 * TRICC_ENOMEM for a short workspace, TRICC_EHIP on a runtime error.
 */
int tricc_core_workspace_size(int32_t n, size_t* bytes);
int tricc_graph_core(const tricc_graph* g, int32_t k_stop, int32_t* d_core, void* d_ws, size_t ws_bytes,
                     int32_t* h_max_core, void* stream);

/*
 * Degeneracy ordering (the k-core row of the paper's Section 4 table of
 * analytics methods, with the Batagelj-Zaversnik decomposition of
 * Section 5). The full core decomposition of tricc_graph_core, which also
 * records for every node the round in which the peeling removed it (every
 * frontier is one round, counted across levels): d_order[v] = that round.
 * A node removed in round r has at most core(v) neighbours removed in round
 * r or later, so the orientation by (d_order[v], v) gives every node an
 * out-degree of at most its core number, and the largest out-degree is at
 * most the degeneracy (the largest core number), against sqrt(2m) for the
 * degree order.
 *   d_order, d_core  device int32[n], the caller's (written)
 *   d_ws, ws_bytes   as for tricc_graph_core
 *   h_degeneracy     host int32 (may be NULL): the largest core number
 * Synchronises `stream`. Errors as tricc_graph_core.
 */
int tricc_graph_degeneracy(const tricc_graph* g, int32_t* d_order, int32_t* d_core, void* d_ws, size_t ws_bytes,
                           int32_t* h_degeneracy, void* stream);

/*
 * Re-orients the graph's DAG by the rank (d_key[v], v) instead of (d(v), v)
 * and re-bins its nodes (steps a4-a5 again on the built simple graph), so
 * that the triangle and 4-clique counts run on that orientation; d_key =
 * NULL restores the degree order. Any strict order gives the same counts;
 * the order only moves work between nodes (with the degeneracy order of
 * tricc_graph_degeneracy, out-degrees are bounded by core numbers).
 *   d_key  device int32[n] of values >= 0 (not checked), or NULL; only read
 *          during the call
 * Clears the statistics of tricc_graph_stats. Synchronises `stream`.
 * Errors: TRICC_EINVAL for a null handle, TRICC_EHIP on a runtime error;
 * TRICC_EINVAL if the graph's tuning cannot hold the new out-degrees (the
 * graph then keeps the new DAG with the old bins unusable: re-orient or
 * retune before counting).
 */
int tricc_graph_reorient(tricc_graph* g, const int32_t* d_key, void* stream);

/*
 * Number of 4-cliques (clique detection, among the graph-motif methods of
 * the paper's Section 4: the triangle count one size up). Counted on the
 * degree-ordered DAG: a 4-clique u < w < x < z (by rank) is met once, at u,
 * from C = N+(u) ∩ N+(w) and the edges x -> z inside C.
 *   d_total   device uint64[1], the caller's (overwritten)
 * Asynchronous on `stream`. Errors: TRICC_EINVAL for a null handle or
 * output; TRICC_EOVERFLOW when some out-degree d+(v) exceeds 8192 (the
 * positions one node's bit rows can index in LDS, one block of them per
 * pass). tricc_graph_reorient with the degeneracy order bounds d+ by the
 * core numbers, which can bring a graph under the limit.
 */
int tricc_graph_count_k4(const tricc_graph* g, uint64_t* d_total, void* stream);

/*
 * Number of 5-cliques (clique detection, as for tricc_graph_count_k4, one
 * size up): a 5-clique u < w < x < y < z (by rank) is met once, at u, from
 * the subgraph induced on N+(u) (bit rows in LDS): x in row w, y in the AND
 * of rows w and x, z in that AND with row y.
 *   d_total   device uint64[1], the caller's (overwritten)
 * Asynchronous on `stream`. Errors: TRICC_EINVAL for a null handle or
 * output; TRICC_EOVERFLOW when some out-degree d+(v) exceeds 1024 (one
 * node's whole bit rows must fit in LDS).
 */
int tricc_graph_count_k5(const tricc_graph* g, uint64_t* d_total, void* stream);

void tricc_graph_free(tricc_graph* g);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation). The
 * same result as tricc_graph_build with the default tuning followed by
 * tricc_count, for a graph of at most TRICC_NOALLOC_MAX_NODES nodes and
 * TRICC_NOALLOC_MAX_PAIRS input pairs, with the graph's workspace taken from
 * a fixed device array of TRICC_NOALLOC_SCRATCH_BYTES inside the library
 * (one per GPU, held until the process ends) instead of a caller buffer.
 * No device or host memory is allocated; the outputs are the caller's, as
 * in tricc_count. Synchronises `stream` (the build reads sizes back).
 * Every call on one GPU uses that GPU's one array, so calls that overlap in
 * time on one GPU (from several threads or streams) race and must not be
 * made; each call clears what it needs before use.
 * Errors: TRICC_EOVERFLOW above the size limits, TRICC_ERANGE for an id
 * outside [0, n), TRICC_EINVAL for null arrays, TRICC_EHIP on a runtime
 * error.
 */
#define TRICC_NOALLOC_MAX_NODES 65536
#define TRICC_NOALLOC_MAX_PAIRS (1LL << 20)
#define TRICC_NOALLOC_SCRATCH_BYTES (32u << 20)
int tricc_count_noalloc(int32_t n, int64_t m_raw, const int32_t* d_src, const int32_t* d_dst, uint64_t* d_node_tri,
                        float* d_node_cc, uint64_t* d_total, double* d_avg_cc, void* stream);

/* ---------------------------------------------------------------------------
 * Batched graphs: many independent graphs counted by one persistent launch.
 *
 * The batch is G graphs packed back to back: graph g has nodes with local
 * ids [0, n_g) and its input pairs at positions [h_edge_off[g],
 * h_edge_off[g+1]) of d_src / d_dst (local ids). h_node_off is the prefix
 * of the n_g (h_node_off[0] = 0, h_node_off[G] = total nodes). Each graph
 * gets the same definitions as a single graph (top of this file); node v of
 * graph g is position h_node_off[g] + v of the per-node outputs.
 */
typedef struct tricc_batch tricc_batch;

typedef struct tricc_batch_tuning {
  int32_t merge_limit;     /* nodes with d+ <= merge_limit take the short-list path (0..wave_limit;
                              at most 16 with variants 2, 3, 6, 7, 32 with 4, 8 with 5) */
  int32_t wave_limit;      /* other nodes with d+ <= wave_limit: one wavefront each (2..64) */
  int32_t persist_variant; /* block nodes up to d+ 256 (0, 2, 4, 5, 6) or 1024 (1, 3, 7);
                              short-list path: 8-lane two-pointer merge (0, 1) or several nodes
                              per wavefront with LDS tables and packed streaming (2..7);
                              cuckoo tables (6, 7) or bucket tables */
  int32_t blocks_per_cu;   /* persistent grid = compute units x this; 0 = occupancy limit */
} tricc_batch_tuning;

typedef struct tricc_batch_info {
  int32_t num_graphs;
  int64_t total_nodes;
  int64_t total_pairs;
  int64_t m;                  /* undirected simple edges over all graphs */
  int64_t max_outdeg;
  int64_t merge_nodes, wave_nodes, block_nodes; /* the persistent kernel's lists */
  int64_t hub_nodes;          /* nodes above the block table: large-table kernels and the fallback */
  int32_t grid;               /* persistent blocks */
  int32_t planned;            /* a hipGraph is instantiated */
} tricc_batch_info;

int tricc_batch_default_tuning(tricc_batch_tuning* out);
int tricc_batch_workspace_size(int32_t num_graphs, int64_t total_nodes, int64_t total_pairs, size_t* bytes);

/* Builds the disjoint union of the batch on the device (validate, map local
 * to global ids, then the a1..a5 build of a single graph) and bins its nodes
 * for the persistent kernel. h_node_off / h_edge_off: host int64[G+1].
 * Synchronises `stream`. TRICC_ERANGE if a local id is outside [0, n_g). */
int tricc_batch_build(int32_t num_graphs, const int64_t* h_node_off, const int64_t* h_edge_off,
                      const int32_t* d_src, const int32_t* d_dst, void* d_ws, size_t ws_bytes,
                      const tricc_batch_tuning* tuning, void* stream, tricc_batch** out);

/* The same batch handed over as a packed CSR (the paper's sorted
 * neighbour vectors, Section 5.1, for each graph, laid end to end): node v of
 * graph g is row h_node_off[g] + v, its entries d_col[d_rowptr[r] ..
 * d_rowptr[r+1]) hold local ids in [0, n_g).
 *   h_node_off  host int64[G+1] as for tricc_batch_build
 *   nnz         entries (d_rowptr[total nodes] must equal it; <= 2^30)
 *   d_rowptr    device int64[total nodes + 1], from 0, non-decreasing
 *   d_col       device int32[nnz]
 *   assume_simple_sorted_symmetric  as for tricc_graph_from_csr: 1 skips the
 *               sort (rows strictly ascending, no self loop, symmetric in
 *               each graph; checked except symmetry), 0 takes every entry as
 *               a pair through the full build
 * Synchronises `stream`. Errors: TRICC_ERANGE for a local id outside its
 * graph's range (or, with 1, outside [0, n)), TRICC_EINVAL for malformed
 * offsets or rows, TRICC_ENOMEM for a short workspace
 * (tricc_batch_workspace_size(G, total nodes, nnz)). */
int tricc_batch_build_csr(int32_t num_graphs, const int64_t* h_node_off, int64_t nnz, const int64_t* d_rowptr,
                          const int32_t* d_col, int assume_simple_sorted_symmetric, void* d_ws, size_t ws_bytes,
                          const tricc_batch_tuning* tuning, void* stream, tricc_batch** out);

/* Binds the outputs and captures the count into a hipGraph: clear (a
 * kernel), the persistent intersection kernel, the per-graph epilogue.
 *   d_node_tri  device uint64[total_nodes] (per-node counts; also the
 *               kernel's accumulator)
 *   d_node_cc   device float[total_nodes]
 *   d_graph_tri device uint64[G]   triangles of each graph
 *   d_graph_avg device double[G]   average CC of each graph over its n_g
 *               nodes, summed in a fixed order that depends only on the graph
 *   d_batch_tri device uint64[1] or NULL: triangles of the whole batch as the
 *               intersection kernels found them, accumulated apart from the
 *               per-node counts (it equals the sum of d_graph_tri when both
 *               are right)
 * The buffers must stay valid while the plan is used. Synchronises. */
int tricc_batch_plan(tricc_batch* b, uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_graph_tri,
                     double* d_graph_avg, uint64_t* d_batch_tri, void* stream);

/* Binds the outputs without capturing a graph (for tricc_batch_run_eager
 * only; a later tricc_batch_plan rebinds). Same buffers as tricc_batch_plan. */
int tricc_batch_bind(tricc_batch* b, uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_graph_tri,
                     double* d_graph_avg, uint64_t* d_batch_tri);

/* One hipGraphLaunch of the planned count. Asynchronous. Calls on one
 * batch must not overlap (they share the accumulators). */
int tricc_batch_run(tricc_batch* b, void* stream);

/* The same three kernels launched directly (no graph). Asynchronous. */
int tricc_batch_run_eager(tricc_batch* b, void* stream);

/* New tuning: re-bins and drops the plan (plan again before running).
 * Synchronises. */
int tricc_batch_retune(tricc_batch* b, const tricc_batch_tuning* tuning, void* stream);

int tricc_batch_info_get(const tricc_batch* b, tricc_batch_info* out);

/* The union graph (for inspection or for counting it with tricc_count). */
const tricc_graph* tricc_batch_graph(const tricc_batch* b);

void tricc_batch_free(tricc_batch* b);

/* ---------------------------------------------------------------------------
 * Query server: triangle count and average clustering coefficient of
 * induced subgraphs G[S] of a graph resident on the device (subgraph
 * extraction, Section 4's table of methods; ids keep their identity,
 * Section 3.1). Degrees are taken inside G[S] and the average is over |S|.
 *
 * The server runs `slots` worker threads, each with its own HIP stream and
 * an equal slice of the caller's device workspace. A worker takes every
 * waiting query that fits its slice (arrival order, at most
 * max_batch_queries) and runs extraction, build and count for them as one
 * batch; queries that arrive meanwhile are taken by the next free worker
 * (continuous batching), and the workers' device work overlaps. A query's
 * result does not depend on which other queries share its batch.
 */
typedef struct tricc_server tricc_server;

typedef struct tricc_result {
  uint64_t qid;
  int64_t k;            /* |S| */
  uint64_t triangles;   /* triangles of G[S] */
  double avg_cc;        /* (1/|S|) sum over S of CC in G[S] (FP64, fixed order) */
  int64_t m;            /* edges of G[S] */
  double t_arrival;     /* as submitted (server clock, seconds) */
  double t_start;       /* batch start */
  double t_done;        /* results on the host */
  int32_t batch_size;   /* queries in the same batch */
  int32_t status;       /* TRICC_OK or the error of the batch */
} tricc_result;

/* `resident` must outlive the server. d_ws / ws_bytes: device workspace,
 * split into `slots` equal slices (1..16); it is also the admission budget:
 * the sum of the admitted, unfinished queries' device bytes never exceeds
 * ws_bytes. Starts the workers. */
int tricc_server_create(const tricc_graph* resident, void* d_ws, size_t ws_bytes, int32_t slots,
                        int32_t max_batch_queries, tricc_server** out);

/* Batch tuning for batches started after this call (default: the batch
 * default). Thread-safe. */
int tricc_server_set_tuning(tricc_server* s, const tricc_batch_tuning* tuning);

/* Seconds since the server was created (steady clock). */
double tricc_server_now(const tricc_server* s);

/* Device bytes a query would need (its admission cost); 0 on bad input. */
size_t tricc_server_query_bytes(const tricc_server* s, const int32_t* h_nodes, int64_t k);

/* Admits query (qid, S = h_nodes[0..k)) with arrival time t_arrival (server
 * clock). The node list is copied. Errors: TRICC_EBUSY when the memory
 * budget is in use (retry after results come back), TRICC_ENOMEM when the
 * query can never fit one slot, TRICC_ERANGE / TRICC_EINVAL for ids outside
 * [0, n) or repeated ids. Thread-safe. */
int tricc_server_submit(tricc_server* s, uint64_t qid, const int32_t* h_nodes, int64_t k, double t_arrival);

/* Moves up to `cap` finished results into out; *n_out = how many. */
int tricc_server_poll(tricc_server* s, tricc_result* out, int32_t cap, int32_t* n_out);

/* Blocks until every admitted query has finished; returns the first batch
 * error, if any. */
int tricc_server_drain(tricc_server* s);

int tricc_server_stats(const tricc_server* s, int64_t* waiting, int64_t* in_flight, size_t* outstanding_bytes);

/* Error text of the calling thread's last failed server call. */
const char* tricc_server_last_error(void);

/* Stops the workers (after the queries in progress) and frees the server. */
void tricc_server_free(tricc_server* s);

#ifdef __cplusplus
}
#endif

#endif /* TRICC_H_ */

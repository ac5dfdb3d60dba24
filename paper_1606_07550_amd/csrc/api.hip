// C ABI of the library: workspace layout, the graph build sequence (steps
// a1..a5), the count sequence (a6..a7) and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/tricc.h"
#include "kernels.h"

using namespace tricc;

namespace {

thread_local char g_err[512] = "";

int fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return status;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(TRICC_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),       \
                  __FILE__, __LINE__);                                                     \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Header words (int32 unless stated).
enum : int {
  kHdrErr = 0,
  kHdrStats = 4,      // [0] max d, [1] max d+
  kHdrDeg2 = 6,       // nodes with d >= 2
  kHdrBinCnt = 16,    // [kNumBins]
  kHdrLimits = 24,    // [kNumBins - 1]
  kHdrListElems = 32, // u64 at byte 128
  kHdrClsOff = 64,    // int64[kNumRowClasses + 1] at byte 256
  kHdrBinOff = 96,    // int64[kNumBins + 1] at byte 384
  kHdrBinElems = 128, // u64[kNumBins] at byte 512
  kHdrBinEdges = 140, // u64[kNumBins] at byte 560, right after the elems
  kHdrInOff = 160,    // int64[kNumBins + 1] at byte 640: in-list bin boundaries
  kHdrInCap = 176,    // int32[kNumBins] at byte 704: chunk size of each bin
  kHdrInItems = 184,  // int64[kNumBins + 1] at byte 736: chunk prefix at the boundaries
  kHdrCheck = 200,    // u64[2] at byte 800: the last count's total and sum of T(v)
  kHdrBinKBytes = 208, // u64[kNumBins] at byte 832: modelled kernel bytes per bin
};
constexpr size_t kHdrBytes = 1024;

struct Layout {
  size_t hdr, raw_off, len, deg, dplus, doff, scan_tmp, rowlist, binlist, adj, tmp, dcol, part_cc,
      part_T, meta, cls_hist, cls_off, din, dinoff, dincol, inlist, inch, incoff, part, hubmap, rec, tot,
      total;
  int64_t cls_nblk;
  int64_t max_jobs;
};

Layout make_layout(int64_t n, int64_t m_raw) {
  Layout L{};
  size_t p = 0;
  auto take = [&](size_t bytes) { size_t at = p; p = align_up(p + std::max<size_t>(bytes, 1)); return at; };
  L.max_jobs = 4 * m_raw / kLargeChunk + 16;
  L.hdr = take(kHdrBytes);
  L.raw_off = take(sizeof(int64_t) * (n + 1));
  L.len = take(sizeof(int32_t) * n);
  L.deg = take(sizeof(int32_t) * n);
  L.dplus = take(sizeof(int32_t) * n);
  L.doff = take(sizeof(int64_t) * (n + 1));
  L.cls_nblk = classify_blocks(n) > 0 ? classify_blocks(n) : 1;
  const int64_t cls_elems = (int64_t)kNumRowClasses * L.cls_nblk;
  L.scan_tmp = take(sizeof(int64_t) * std::max(scan_tmp_elems(n + 1), scan_tmp_elems(cls_elems + 1)));
  L.cls_hist = take(sizeof(int32_t) * cls_elems);
  L.cls_off = take(sizeof(int64_t) * (cls_elems + 1));
  L.rowlist = take(sizeof(int32_t) * n);
  L.binlist = take(sizeof(int32_t) * n);
  L.adj = take(sizeof(int32_t) * 2 * m_raw);
  L.tmp = take(sizeof(int32_t) * 2 * m_raw);
  L.dcol = take(sizeof(int32_t) * m_raw + 16);  // 16-byte loads may run 3 ids past the end
  L.part_cc = take(sizeof(double) * epilogue_blocks(n));
  L.part_T = take(sizeof(unsigned long long) * epilogue_blocks(n));
  L.meta = take(64 * (size_t)L.max_jobs + 4096);
  L.din = take(sizeof(int32_t) * n);
  L.dinoff = take(sizeof(int64_t) * (n + 1));
  L.dincol = take(sizeof(int32_t) * m_raw + 16);
  L.inlist = take(sizeof(int32_t) * n);
  L.inch = take(sizeof(int32_t) * n);
  L.incoff = take(sizeof(int64_t) * (n + 1));
  L.part = take(2 * sizeof(uint32_t) * kPartMaxParts + 2 * sizeof(int64_t) * (kPartMaxParts + 1));
  L.hubmap = take(sizeof(uint32_t) * (size_t)hub_map_words(n) * (size_t)hub_map_slots(n));
  L.rec = take(sizeof(int32_t) * 2 * n);  // edge-existence records (row start, degree)
  L.tot = take(sizeof(unsigned long long) * kTotSlots);  // triangle-total counters
  L.total = p;
  return L;
}

}  // namespace

struct tricc_graph {
  int32_t n;
  int64_t m_raw;
  char* ws;
  Layout L;
  hipStream_t stream;
  tricc_tuning tuning;
  tricc_graph_info info;
  int64_t bin_off[kNumBins + 1];
  int64_t in_off[kNumBins + 1];    // in-list nodes of each bin (min-side)
  int64_t in_items[kNumBins + 1];  // chunk prefix at the in-list bin boundaries
  int64_t cls_off[kNumRowClasses + 1];  // row classes (by raw length) in the row list
  int32_t oriented_by_key;         // 1 when the DAG follows a caller's key, not the degrees
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  int32_t* hdr32() const { return at<int32_t>(L.hdr); }
};

namespace {

int sync_copy(void* h, const void* d, size_t bytes, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return TRICC_OK;
}

int upload(void* d, const void* h, size_t bytes, hipStream_t s) {
  if (!bytes) return TRICC_OK;
  HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return TRICC_OK;
}

void tricc_default_tuning_impl(tricc_tuning* out);

int check_tuning(const tricc_tuning* t) {
  for (int b = 0; b < kNumBins; ++b)
    if (!count_variant_valid(t->bin_variant[b]))
      return fail(TRICC_EINVAL, "tuning: bin %d has unknown variant %d", b, t->bin_variant[b]);
  for (int b = 0; b < kNumBins - 1; ++b)
    if (t->bin_limit[b] < 0) return fail(TRICC_EINVAL, "tuning: negative bin limit");
  if (t->min_side != 0 && t->min_side != 1) return fail(TRICC_EINVAL, "tuning: min_side must be 0 or 1");
  if (t->min_side)
    for (int b = 0; b < kNumBins - 1; ++b)
      if (!count_variant_min_side(t->bin_variant[b]))
        return fail(TRICC_EINVAL, "tuning: min_side needs min-side variants in bins 0..4 (bin %d has %d)", b,
                    t->bin_variant[b]);
  return TRICC_OK;
}

// Large rows (> kLargeChunk entries): sort chunks in LDS, merge runs pairwise
// between adj and tmp, then dedup into adj.
int sort_large_rows(tricc_graph* g, int32_t nl, const int32_t* rows_dev) {
  hipStream_t s = g->stream;
  const Layout& L = g->L;
  char* meta = g->ws + L.meta;
  int64_t* d_off = reinterpret_cast<int64_t*>(meta);
  int32_t* d_len = reinterpret_cast<int32_t*>(meta + align_up(sizeof(int64_t) * nl));
  HIPCHK(launch_gather_rows(rows_dev, nl, g->at<int64_t>(L.raw_off), g->at<int32_t>(L.len), d_off, d_len, s));
  std::vector<int64_t> h_off(nl), tmp_beg(nl);
  std::vector<int32_t> h_len(nl);
  int rc = sync_copy(h_off.data(), d_off, sizeof(int64_t) * nl, s);
  if (rc) return rc;
  if ((rc = sync_copy(h_len.data(), d_len, sizeof(int32_t) * nl, s))) return rc;
  int64_t acc = 0;
  int32_t maxL = 0;
  for (int i = 0; i < nl; ++i) { tmp_beg[i] = acc; acc += h_len[i]; maxL = std::max(maxL, h_len[i]); }
  int32_t* adj = g->at<int32_t>(L.adj);
  int32_t* tmp = g->at<int32_t>(L.tmp);

  std::vector<int64_t> cbeg;
  std::vector<int32_t> clen;
  for (int i = 0; i < nl; ++i)
    for (int64_t c = 0; c < h_len[i]; c += kLargeChunk) {
      cbeg.push_back(h_off[i] + c);
      clen.push_back((int32_t)std::min<int64_t>(kLargeChunk, h_len[i] - c));
    }
  const int64_t nj_max = (int64_t)cbeg.size();
  if (nj_max > L.max_jobs) return fail(TRICC_EOVERFLOW, "too many large-row chunks");
  // The job arrays of a step (chunk sort, each merge pass, the dedup) sit in
  // one block of meta, int64 arrays first, and go up in one copy: a pass has
  // at most nj_max jobs (each covers 2 R >= 2 chunks of a row), and the
  // block is rewritten only after the previous step's kernel (stream order).
  int64_t* m_a = reinterpret_cast<int64_t*>(meta);
  int64_t* m_o = m_a + nj_max;
  int64_t* m_t = m_o + nj_max;
  int32_t* m_la = reinterpret_cast<int32_t*>(m_t + nj_max + 1);
  int32_t* m_lb = m_la + nj_max;
  std::vector<int64_t> blk((size_t)(3 * nj_max + 1) + (size_t)(nj_max + 1));  // int64 view of the block
  int32_t* blk32 = reinterpret_cast<int32_t*>(blk.data() + 3 * nj_max + 1);
  std::copy(cbeg.begin(), cbeg.end(), blk.begin());
  std::copy(clen.begin(), clen.end(), blk32);
  if ((rc = upload(m_a, blk.data(), sizeof(int64_t) * blk.size(), s))) return rc;
  HIPCHK(launch_sort_chunks(m_a, m_la, (int32_t)nj_max, adj, s));

  bool in_adj = true;
  for (int64_t R = kLargeChunk; R < maxL; R *= 2) {
    std::vector<int64_t> a, o, t;
    std::vector<int32_t> la, lb;
    int64_t tiles = 0;
    for (int i = 0; i < nl; ++i) {
      const int64_t Li = h_len[i];
      const int64_t bin = in_adj ? h_off[i] : tmp_beg[i];
      const int64_t bout = in_adj ? tmp_beg[i] : h_off[i];
      for (int64_t k = 0; k < Li; k += 2 * R) {
        const int64_t A = std::min(R, Li - k);
        const int64_t B = std::max<int64_t>(0, std::min(R, Li - k - R));
        a.push_back(bin + k);
        o.push_back(bout + k);
        la.push_back((int32_t)A);
        lb.push_back((int32_t)B);
        t.push_back(tiles);
        tiles += (A + B + kMergeTile - 1) / kMergeTile;
      }
    }
    t.push_back(tiles);
    const int32_t nj = (int32_t)a.size();
    if (nj > nj_max) return fail(TRICC_EOVERFLOW, "merge pass with more jobs than chunks");
    std::copy(a.begin(), a.end(), blk.begin());
    std::copy(o.begin(), o.end(), blk.begin() + nj_max);
    std::copy(t.begin(), t.end(), blk.begin() + 2 * nj_max);
    std::copy(la.begin(), la.end(), blk32);
    std::copy(lb.begin(), lb.end(), blk32 + nj_max);
    if ((rc = upload(m_a, blk.data(), sizeof(int64_t) * blk.size(), s))) return rc;
    HIPCHK(launch_merge_pass(m_a, m_la, m_lb, m_o, m_t, nj, tiles, in_adj ? adj : tmp, in_adj ? tmp : adj, s));
    in_adj = !in_adj;
  }
  std::vector<int64_t> seg(nl);
  for (int i = 0; i < nl; ++i) seg[i] = in_adj ? h_off[i] : tmp_beg[i];
  if ((rc = upload(m_a, seg.data(), sizeof(int64_t) * nl, s))) return rc;
  HIPCHK(launch_dedup_rows(rows_dev, m_a, nl, g->at<int32_t>(L.len), in_adj ? adj : tmp,
                           g->at<int64_t>(L.raw_off), adj, g->at<int32_t>(L.deg), s));
  g->info.large_rows = nl;
  return TRICC_OK;
}

// Runs a two-pass classification; h_off receives nc + 1 class offsets.
template <typename Launch>
int classify(tricc_graph* g, int nc, Launch launch, int64_t* d_cls_off, int64_t* h_off) {
  hipStream_t s = g->stream;
  const Layout& L = g->L;
  int32_t* hist = g->at<int32_t>(L.cls_hist);
  int64_t* off = g->at<int64_t>(L.cls_off);
  HIPCHK(launch(0, hist, off));
  HIPCHK(launch_scan_i32(hist, (int64_t)nc * L.cls_nblk, off, g->at<int64_t>(L.scan_tmp), s));
  HIPCHK(launch_class_offsets(off, L.cls_nblk, nc, d_cls_off, s));
  HIPCHK(launch(1, hist, off));
  return sync_copy(h_off, d_cls_off, sizeof(int64_t) * (nc + 1), s);
}

int bin_nodes(tricc_graph* g) {
  hipStream_t s = g->stream;
  const Layout& L = g->L;
  int32_t* hdr = g->hdr32();
  const int32_t n = g->n;
  int rc = upload(hdr + kHdrLimits, g->tuning.bin_limit, sizeof(int32_t) * (kNumBins - 1), s);
  if (rc) return rc;
  int64_t* d_bin_off = reinterpret_cast<int64_t*>(g->ws + L.hdr + kHdrBinOff * 4);
  const int32_t* dplus = g->at<int32_t>(L.dplus);
  int32_t* binlist = g->at<int32_t>(L.binlist);
  auto launch = [&](int pass, int32_t* hist, const int64_t* off) {
    return launch_classify_bins(pass, n, dplus, hdr + kHdrLimits, hist, off, L.cls_nblk, binlist, s);
  };
  if (n == 0) {
    for (int b = 0; b <= kNumBins; ++b) g->bin_off[b] = 0;
  } else if ((rc = classify(g, kNumBins, launch, d_bin_off, g->bin_off))) {
    return rc;
  }
  for (int b = 0; b < kNumBins; ++b) {
    const int64_t cnt = g->bin_off[b + 1] - g->bin_off[b];
    g->info.bin_count[b] = cnt;
    g->info.bin_list_elems[b] = 0;
    g->info.bin_edges[b] = 0;
    g->info.bin_kernel_bytes[b] = 0;
    if (!cnt) continue;
    int64_t bound = g->info.max_outdeg;
    if (b < kNumBins - 1) bound = std::min<int64_t>(bound, g->tuning.bin_limit[b]);
    const int cap = count_variant_capacity(g->tuning.bin_variant[b]);
    if (cap < bound)
      return fail(TRICC_EINVAL, "tuning: bin %d holds out-degrees up to %lld but variant %d accepts %d", b,
                  (long long)bound, g->tuning.bin_variant[b], cap);
  }
  g->info.list_elems = 0;
  // in-list items (min-side): owners by d+(w), chunks of the bin variant's capacity
  for (int b = 0; b <= kNumBins; ++b) g->in_off[b] = g->in_items[b] = 0;
  if (g->tuning.min_side && n > 0) {
    int64_t* d_in_off = reinterpret_cast<int64_t*>(g->ws + L.hdr + kHdrInOff * 4);
    int32_t* inlist = g->at<int32_t>(L.inlist);
    auto launch_in = [&](int pass, int32_t* hist, const int64_t* off) {
      return launch_classify_inbins(pass, n, dplus, g->at<int32_t>(L.deg), hdr + kHdrLimits, hist, off, L.cls_nblk,
                                    inlist, s);
    };
    if ((rc = classify(g, kNumBins, launch_in, d_in_off, g->in_off))) return rc;
    int32_t caps[kNumBins];
    for (int b = 0; b < kNumBins; ++b) caps[b] = std::max(1, std::min(1 << 20, count_variant_capacity(g->tuning.bin_variant[b])));
    if ((rc = upload(hdr + kHdrInCap, caps, sizeof(caps), s))) return rc;
    const int64_t nin = g->in_off[kNumBins];
    HIPCHK(launch_in_chunks(inlist, nin, g->at<int32_t>(L.din), hdr + kHdrInCap, d_in_off, g->at<int32_t>(L.inch), s));
    int64_t* incoff = g->at<int64_t>(L.incoff);
    HIPCHK(launch_scan_i32(g->at<int32_t>(L.inch), nin, incoff, g->at<int64_t>(L.scan_tmp), s));
    // chunk -> owner map in tmp (free after the orientation): at most one
    // chunk per owner plus d-(w) / 16 per owner, below the 2 m_raw entries
    HIPCHK(launch_in_owners(nin, incoff, g->at<int32_t>(L.tmp), s));
    int64_t* d_items = reinterpret_cast<int64_t*>(g->ws + L.hdr + kHdrInItems * 4);
    HIPCHK(launch_gather_offsets(incoff, d_in_off, kNumBins + 1, d_items, s));
    if ((rc = sync_copy(g->in_items, d_items, sizeof(g->in_items), s))) return rc;
  }
  for (int b = 0; b < kNumBins; ++b) g->info.bin_in_items[b] = g->in_items[b + 1] - g->in_items[b];
  return TRICC_OK;
}

// Algorithmic-size statistics (not needed for counting).
int graph_stats(tricc_graph* g) {
  hipStream_t s = g->stream;
  const Layout& L = g->L;
  unsigned long long* d_elems = reinterpret_cast<unsigned long long*>(g->ws + L.hdr + kHdrBinElems * 4);
  unsigned long long* d_edges = reinterpret_cast<unsigned long long*>(g->ws + L.hdr + kHdrBinEdges * 4);
  unsigned long long* d_all = reinterpret_cast<unsigned long long*>(g->ws + L.hdr + kHdrListElems * 4);
  unsigned long long* d_kb = reinterpret_cast<unsigned long long*>(g->ws + L.hdr + kHdrBinKBytes * 4);
  HIPCHK(hipMemsetAsync(d_elems, 0, sizeof(unsigned long long) * 2 * kNumBins, s));
  HIPCHK(hipMemsetAsync(d_kb, 0, sizeof(unsigned long long) * kNumBins, s));
  HIPCHK(hipMemsetAsync(d_all, 0, sizeof(unsigned long long), s));
  HIPCHK(launch_bin_elems(g->n, g->at<int64_t>(L.doff), g->at<int32_t>(L.dcol), g->at<int32_t>(L.din),
                          g->hdr32() + kHdrLimits, g->hdr32() + kHdrInCap,
                          g->tuning.min_side ? g->tuning.bin_limit[kNumBins - 2] : 0, d_elems, d_edges, d_kb, s));
  HIPCHK(launch_list_elems(g->n, g->at<int64_t>(L.doff), g->at<int32_t>(L.dcol), d_all, s));
  unsigned long long be[2 * kNumBins];
  int rc = sync_copy(be, d_elems, sizeof(be), s);
  if (rc) return rc;
  unsigned long long all = 0, kb[kNumBins];
  if ((rc = sync_copy(&all, d_all, sizeof(all), s))) return rc;
  if ((rc = sync_copy(kb, d_kb, sizeof(kb), s))) return rc;
  for (int b = 0; b < kNumBins; ++b) {
    g->info.bin_list_elems[b] = be[b];
    g->info.bin_edges[b] = (int64_t)be[kNumBins + b];
    g->info.bin_kernel_bytes[b] = kb[b];
  }
  g->info.list_elems = all;
  return TRICC_OK;
}

// a4-a5: orient every edge of the simple graph from the lower to the higher
// rank (key(v), v), with key = the degrees when key is null, then bin the
// DAG's nodes. The simple graph's rows (adj, raw_off, len, deg) and the row
// lists by class are read; the DAG, in-lists, d+, d- and bins are rewritten.
int orient_impl(tricc_graph* g, const int32_t* key) {
  hipStream_t s = g->stream;
  const Layout& L = g->L;
  const int32_t n = g->n;
  int32_t* hdr = g->hdr32();
  int32_t* len = g->at<int32_t>(L.len);
  int32_t* deg = g->at<int32_t>(L.deg);
  int64_t* raw_off = g->at<int64_t>(L.raw_off);
  int64_t* scan_tmp = g->at<int64_t>(L.scan_tmp);
  int32_t* adj = g->at<int32_t>(L.adj);
  int32_t* rowlist = g->at<int32_t>(L.rowlist);
  const int64_t* cls_off = g->cls_off;
  int rc;
  HIPCHK(hipMemsetAsync(hdr + kHdrStats, 0, sizeof(int32_t) * 3, s));  // max d, max d+, nodes with d >= 2
  // a4: orientation (rows longer than 64 raw entries: classes kRow128 ..
  // kRowLds4k are medium, the classes above them are long; the row lists
  // are class-major, so each range is contiguous)
  int32_t* dplus = g->at<int32_t>(L.dplus);
  int64_t* doff = g->at<int64_t>(L.doff);
  int32_t* dcol = g->at<int32_t>(L.dcol);
  const int32_t* med_rows = rowlist + cls_off[kRow128];
  const int32_t nmed = (int32_t)(cls_off[kRowLds4k + 1] - cls_off[kRow128]);
  const int32_t* long_rows = rowlist + cls_off[kRowLds8k];
  const int32_t nlong = (int32_t)(cls_off[kNumRowClasses] - cls_off[kRowLds8k]);
  // one pass partitions every row into tmp (free again after a3), then
  // the scans place the out- and in-lists
  int32_t* part = g->at<int32_t>(L.tmp);
  // the degree-class words (n / 4 bytes) sit in binlist, free until the binning
  uint32_t* cls = reinterpret_cast<uint32_t*>(g->at<int32_t>(L.binlist));
  HIPCHK(launch_orient(n, raw_off, len, deg, key, adj, med_rows, nmed, long_rows, nlong, cls, dplus, part,
                       hdr + kHdrStats, s));
  HIPCHK(launch_scan_i32(dplus, n, doff, scan_tmp, s));
  int32_t* din = g->at<int32_t>(L.din);
  int64_t* dinoff = g->at<int64_t>(L.dinoff);
  HIPCHK(launch_indeg(n, deg, dplus, din, hdr + kHdrDeg2, s));
  HIPCHK(launch_scan_i32(din, n, dinoff, scan_tmp, s));
  HIPCHK(launch_orient_copy(n, raw_off, len, deg, dplus, part, med_rows, nmed, long_rows, nlong, doff, dcol, dinoff,
                            g->at<int32_t>(L.dincol), s));
  HIPCHK(launch_edge_records(n, raw_off, deg, g->at<int32_t>(L.rec), s));
  int32_t stats[3];  // max d, max d+, nodes with d >= 2
  if ((rc = sync_copy(stats, hdr + kHdrStats, sizeof(stats), s))) return rc;
  int64_t m = 0;
  if ((rc = sync_copy(&m, doff + n, sizeof(m), s))) return rc;
  g->info.m = m;
  g->info.max_deg = stats[0];
  g->info.max_outdeg = stats[1];
  g->info.n_deg2 = stats[2];
  g->oriented_by_key = key != nullptr;
  // a5: binning
  return bin_nodes(g);
}

// Builds a1-a5. With presorted set, adj, raw_off, len and deg already hold
// simple, sorted, symmetric rows (a caller CSR that was checked) and a1-a3
// reduce to the row classification that the orientation needs.
int build_impl(tricc_graph* g, const int32_t* src, const int32_t* dst, bool presorted = false) {
  hipStream_t s = g->stream;
  const Layout& L = g->L;
  const int32_t n = g->n;
  const int64_t m_raw = g->m_raw;
  int32_t* hdr = g->hdr32();
  int32_t* len = g->at<int32_t>(L.len);
  int32_t* deg = g->at<int32_t>(L.deg);
  int64_t* raw_off = g->at<int64_t>(L.raw_off);
  int64_t* scan_tmp = g->at<int64_t>(L.scan_tmp);
  int32_t* adj = g->at<int32_t>(L.adj);
  int rc;

  // the hub variant expects zeroed bitmaps and leaves them zeroed
  HIPCHK(hipMemsetAsync(g->ws + L.hubmap, 0, sizeof(uint32_t) * (size_t)hub_map_words(n) * hub_map_slots(n), s));
  if (!presorted) HIPCHK(hipMemsetAsync(hdr, 0, kHdrBytes, s));
  if (!presorted) HIPCHK(hipMemsetAsync(len, 0, sizeof(int32_t) * (size_t)n, s));
  const int pbits = m_raw > 0 && !presorted ? part_bits(n) : -1;
  int32_t err = 0;
  if (presorted) {
    // rows in place
  } else if (pbits >= 0) {
    // a1-a3 partitioned: validate, stage every entry in its partition's
    // slice (other endpoint in tmp, local row in the not yet used dcol
    // area), then raw lengths, row offsets and unsorted rows per partition
    const int32_t P = (int32_t)((n + (int64_t(1) << pbits) - 1) >> pbits);
    uint32_t* ptotal = g->at<uint32_t>(L.part);
    uint32_t* pcur = ptotal + kPartMaxParts;
    int64_t* pstart = reinterpret_cast<int64_t*>(pcur + kPartMaxParts);
    int64_t* cstart = pstart + kPartMaxParts + 1;
    int32_t* pv = g->at<int32_t>(L.tmp);
    uint16_t* pu = g->at<uint16_t>(L.dcol);
    int32_t* cur = g->at<int32_t>(L.binlist);
    HIPCHK(hipMemsetAsync(ptotal, 0, 2 * sizeof(uint32_t) * kPartMaxParts, s));
    HIPCHK(launch_part_count(src, dst, m_raw, n, pbits, P, ptotal, hdr + kHdrErr, s));
    if ((rc = sync_copy(&err, hdr + kHdrErr, sizeof(err), s))) return rc;
    if (err) return fail(TRICC_ERANGE, "edge list holds a node id outside [0, %d)", n);
    HIPCHK(launch_part_scan(ptotal, P, pstart, cstart, s));
    HIPCHK(launch_part_place(src, dst, m_raw, pbits, P, pstart, pcur, pv, pu, s));
    HIPCHK(launch_part_rows(0, pbits, P, n, 2 * m_raw, pstart, cstart, pu, pv, len, raw_off, cur, adj, s));
    HIPCHK(launch_scan_i32(len, n, raw_off, scan_tmp, s));
    HIPCHK(hipMemsetAsync(cur, 0, sizeof(int32_t) * (size_t)n, s));
    HIPCHK(launch_part_rows(1, pbits, P, n, 2 * m_raw, pstart, cstart, pu, pv, len, raw_off, cur, adj, s));
  } else {
    // a1: validate + raw degrees
    HIPCHK(launch_degree_raw(src, dst, m_raw, n, len, hdr + kHdrErr, s));
    if ((rc = sync_copy(&err, hdr + kHdrErr, sizeof(err), s))) return rc;
    if (err) return fail(TRICC_ERANGE, "edge list holds a node id outside [0, %d)", n);
    // a2: row offsets
    HIPCHK(launch_scan_i32(len, n, raw_off, scan_tmp, s));
    HIPCHK(hipMemsetAsync(len, 0, sizeof(int32_t) * (size_t)n, s));
    // a3: scatter (len ends equal to the raw row lengths again)
    HIPCHK(launch_scatter(src, dst, m_raw, raw_off, len, adj, s));
  }
  // a3: row sort and dedup
  int32_t* rowlist = g->at<int32_t>(L.rowlist);
  int64_t* d_cls_off = reinterpret_cast<int64_t*>(g->ws + L.hdr + kHdrClsOff * 4);
  int64_t cls_off[kNumRowClasses + 1] = {};
  if (n > 0) {
    auto launch = [&](int pass, int32_t* hist, const int64_t* off) {
      return launch_classify_rows(pass, n, len, deg, hist, off, L.cls_nblk, rowlist, s);
    };
    if ((rc = classify(g, kNumRowClasses, launch, d_cls_off, cls_off))) return rc;
  }
  int32_t cnt[kNumRowClasses];
  for (int c = 0; c < kNumRowClasses; ++c) cnt[c] = (int32_t)(cls_off[c + 1] - cls_off[c]);
  g->info.large_rows = 0;
  if (!presorted) {
    for (int c = kRow8; c <= kRowLds32k; ++c)
      HIPCHK(launch_sort_rows(c, rowlist + cls_off[c], cnt[c], raw_off, len, adj, deg, s));
    if (cnt[kRowLarge] > 0)
      if ((rc = sort_large_rows(g, cnt[kRowLarge], rowlist + cls_off[kRowLarge]))) return rc;
  }
  for (int c = 0; c <= kNumRowClasses; ++c) g->cls_off[c] = cls_off[c];
  g->info.n = n;
  g->info.m_raw = m_raw;
  return orient_impl(g, nullptr);
}


}  // namespace

namespace {
// a1-a5 from a CSR (see tricc_graph_from_csr); g's size, layout, stream and
// tuning are set. Reads the caller's arrays only.
int csr_build(tricc_graph* g, int64_t nnz, const int64_t* d_rowptr, const int32_t* d_col,
              int assume_simple_sorted_symmetric) {
  const int32_t n = g->n;
  const Layout& L = g->L;
  hipStream_t s = g->stream;
  int32_t* hdr = g->hdr32();
  int32_t err = 0;
  int r;
  HIPCHK(hipMemsetAsync(hdr, 0, kHdrBytes, s));
  if (!assume_simple_sorted_symmetric) {
    // rows as (v, w) pairs through the full build; the pair sources sit in
    // the in-list area, which the build writes only after a3
    HIPCHK(launch_csr_bounds(n, nnz, d_rowptr, nullptr, nullptr, hdr + kHdrErr, s));
    if ((r = sync_copy(&err, hdr + kHdrErr, sizeof(err), s))) return r;
    if (err) return fail(TRICC_EINVAL, "CSR row offsets are not a non-decreasing sequence from 0 to nnz");
    int32_t* src = g->at<int32_t>(L.dincol);
    HIPCHK(launch_csr_expand(n, d_rowptr, src, s));
    return build_impl(g, src, d_col);
  }
  int64_t* raw_off = g->at<int64_t>(L.raw_off);
  int32_t* adj = g->at<int32_t>(L.adj);
  HIPCHK(hipMemcpyAsync(raw_off, d_rowptr, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_csr_bounds(n, nnz, raw_off, g->at<int32_t>(L.len), g->at<int32_t>(L.deg), hdr + kHdrErr, s));
  if ((r = sync_copy(&err, hdr + kHdrErr, sizeof(err), s))) return r;
  if (err) return fail(TRICC_EINVAL, "CSR row offsets are not a non-decreasing sequence from 0 to nnz");
  if (nnz > 0) HIPCHK(hipMemcpyAsync(adj, d_col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_csr_rows(n, raw_off, adj, hdr + kHdrErr, s));
  if ((r = sync_copy(&err, hdr + kHdrErr, sizeof(err), s))) return r;
  if (err & 1) return fail(TRICC_ERANGE, "CSR holds a node id outside [0, %d)", n);
  if (err) return fail(TRICC_EINVAL, "CSR row not strictly ascending or holding its own id");
  return build_impl(g, nullptr, nullptr, true);
}

}  // namespace

namespace {
void tricc_default_tuning_impl(tricc_tuning* out) {
  static const int32_t lim[kNumBins - 1] = {64, 192, 512, 1024, 4096};
  static const int32_t var[kNumBins] = {21, 23, 24, 20, 14, 9};
  std::memcpy(out->bin_limit, lim, sizeof(lim));
  std::memcpy(out->bin_variant, var, sizeof(var));
  out->min_side = 1;
}
}  // namespace

extern "C" {

const char* tricc_status_str(int status) {
  switch (status) {
    case TRICC_OK: return "ok";
    case TRICC_EINVAL: return "invalid argument";
    case TRICC_ERANGE: return "node id out of range";
    case TRICC_ENOMEM: return "workspace or memory budget too small";
    case TRICC_EHIP: return "HIP runtime error";
    case TRICC_EBUSY: return "busy: admission refused";
    case TRICC_EOVERFLOW: return "size not supported";
    default: return "unknown status";
  }
}

const char* tricc_last_error(void) { return g_err; }

int tricc_version(void) { return 100; }

int tricc_default_tuning(tricc_tuning* out) {
  if (!out) return fail(TRICC_EINVAL, "null tuning");
  tricc_default_tuning_impl(out);
  return TRICC_OK;
}

int tricc_variant_capacity(int variant) { return count_variant_capacity(variant); }

int tricc_variant_min_side(int variant) { return count_variant_min_side(variant); }

int tricc_variant_count(void) {
  int v = 0;
  while (count_variant_valid(v)) ++v;
  return v;
}

int tricc_graph_workspace_size(int32_t n, int64_t m_raw, size_t* bytes) {
  if (!bytes) return fail(TRICC_EINVAL, "null bytes");
  if (n < 0 || n >= 0x7fffffff) return fail(TRICC_EINVAL, "n out of range");
  if (m_raw < 0) return fail(TRICC_EINVAL, "m_raw negative");
  if (m_raw > (int64_t(1) << 30)) return fail(TRICC_EOVERFLOW, "m_raw above 2^30");
  *bytes = make_layout(n, m_raw).total;
  return TRICC_OK;
}

int tricc_graph_build(int32_t n, int64_t m_raw, const int32_t* d_src, const int32_t* d_dst, void* d_ws,
                      size_t ws_bytes, const tricc_tuning* tuning, void* stream, tricc_graph** out) {
  g_err[0] = 0;
  if (!out) return fail(TRICC_EINVAL, "null out");
  *out = nullptr;
  size_t need = 0;
  int rc = tricc_graph_workspace_size(n, m_raw, &need);
  if (rc) return rc;
  if (m_raw > 0 && (!d_src || !d_dst)) return fail(TRICC_EINVAL, "null edge arrays");
  if (!d_ws) return fail(TRICC_EINVAL, "null workspace");
  if (ws_bytes < need) return fail(TRICC_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(TRICC_EINVAL, "workspace not 256-byte aligned");
  tricc_tuning t;
  if (tuning) t = *tuning; else tricc_default_tuning(&t);
  if ((rc = check_tuning(&t))) return rc;
  tricc_graph* g = new (std::nothrow) tricc_graph();
  if (!g) return fail(TRICC_ENOMEM, "host allocation failed");
  g->n = n;
  g->m_raw = m_raw;
  g->ws = static_cast<char*>(d_ws);
  g->L = make_layout(n, m_raw);
  g->stream = static_cast<hipStream_t>(stream);
  g->tuning = t;
  std::memset(&g->info, 0, sizeof(g->info));
  rc = build_impl(g, d_src, d_dst);
  if (rc) {
    delete g;
    return rc;
  }
  *out = g;
  return TRICC_OK;
}

int tricc_graph_from_csr(int32_t n, int64_t nnz, const int64_t* d_rowptr, const int32_t* d_col,
                         int assume_simple_sorted_symmetric, void* d_ws, size_t ws_bytes, const tricc_tuning* tuning,
                         void* stream, tricc_graph** out) {
  g_err[0] = 0;
  if (!out) return fail(TRICC_EINVAL, "null out");
  *out = nullptr;
  size_t need = 0;
  int rc = tricc_graph_workspace_size(n, nnz, &need);
  if (rc) return rc;
  if (!d_rowptr || (nnz > 0 && !d_col)) return fail(TRICC_EINVAL, "null CSR arrays");
  if (!d_ws) return fail(TRICC_EINVAL, "null workspace");
  if (ws_bytes < need) return fail(TRICC_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(TRICC_EINVAL, "workspace not 256-byte aligned");
  tricc_tuning t;
  if (tuning) t = *tuning; else tricc_default_tuning(&t);
  if ((rc = check_tuning(&t))) return rc;
  tricc_graph* g = new (std::nothrow) tricc_graph();
  if (!g) return fail(TRICC_ENOMEM, "host allocation failed");
  g->n = n;
  g->m_raw = nnz;
  g->ws = static_cast<char*>(d_ws);
  g->L = make_layout(n, nnz);
  g->stream = static_cast<hipStream_t>(stream);
  g->tuning = t;
  std::memset(&g->info, 0, sizeof(g->info));
  rc = csr_build(g, nnz, d_rowptr, d_col, assume_simple_sorted_symmetric);
  if (rc) {
    delete g;
    return rc;
  }
  *out = g;
  return TRICC_OK;
}

int tricc_graph_info_get(const tricc_graph* g, tricc_graph_info* out) {
  if (!g || !out) return fail(TRICC_EINVAL, "null argument");
  *out = g->info;
  return TRICC_OK;
}

int tricc_graph_stats(tricc_graph* g, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  g->stream = static_cast<hipStream_t>(stream);
  return graph_stats(g);
}

int tricc_graph_retune(tricc_graph* g, const tricc_tuning* tuning, void* stream) {
  if (!g || !tuning) return fail(TRICC_EINVAL, "null argument");
  int rc = check_tuning(tuning);
  if (rc) return rc;
  const tricc_tuning old = g->tuning;
  g->tuning = *tuning;
  g->stream = static_cast<hipStream_t>(stream);
  rc = bin_nodes(g);
  if (rc) {
    g->tuning = old;
    int rc2 = bin_nodes(g);
    (void)rc2;
  }
  return rc;
}

int tricc_count_begin(tricc_graph* g, uint64_t* d_node_tri, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (g->n > 0 && !d_node_tri) return fail(TRICC_EINVAL, "null output");
  HIPCHK(launch_zero_counts(reinterpret_cast<unsigned long long*>(d_node_tri), g->n,
                            g->at<unsigned long long>(g->L.tot), static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

}  // extern "C"

namespace {

// Bins b0 .. b1 (one variant) in one launch: their node lists, in-list
// owners and chunks are contiguous, so the launch covers the union, and the
// last blocks of one bin overlap the next bin's instead of draining first.
int count_bins(tricc_graph* g, int b0, int b1, uint64_t* d_node_tri, void* stream) {
  const int32_t count = (int32_t)(g->bin_off[b1 + 1] - g->bin_off[b0]);
  if (count == 0 && g->in_items[b1 + 1] == g->in_items[b0]) return TRICC_OK;
  if (!d_node_tri) return fail(TRICC_EINVAL, "null output");
  const Layout& L = g->L;
  BinLaunch bl{g->tuning.bin_variant[b0], g->at<int32_t>(L.binlist) + g->bin_off[b0], count};
  if (g->tuning.min_side && count_variant_min_side(bl.variant)) {
    bl.in_list = g->at<int32_t>(L.inlist) + g->in_off[b0];
    bl.in_coff = g->at<int64_t>(L.incoff) + g->in_off[b0];
    bl.in_owner = g->at<int32_t>(L.tmp) + g->in_items[b0];
    bl.in_base = (int32_t)g->in_off[b0];
    bl.in_nodes = (int32_t)(g->in_off[b1 + 1] - g->in_off[b0]);
    bl.in_items = g->in_items[b1 + 1] - g->in_items[b0];
    bl.w_max = g->tuning.bin_limit[kNumBins - 2];
    bl.dinoff = g->at<int64_t>(L.dinoff);
    bl.dincol = g->at<int32_t>(L.dincol);
  }
  bl.hubmap = g->at<uint32_t>(L.hubmap);
  bl.hub_slots = hub_map_slots(g->n);
  bl.map_words = hub_map_words(g->n);
  HIPCHK(launch_count_bin(bl, g->at<int64_t>(L.doff), g->at<int32_t>(L.dcol),
                          reinterpret_cast<unsigned long long*>(d_node_tri), g->at<unsigned long long>(L.tot),
                          static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

}  // namespace

extern "C" {

int tricc_count_bin(tricc_graph* g, int bin, uint64_t* d_node_tri, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (bin < 0 || bin >= kNumBins) return fail(TRICC_EINVAL, "bin %d out of range", bin);
  return count_bins(g, bin, bin, d_node_tri, stream);
}

int tricc_count_bins(tricc_graph* g, int first, int last, uint64_t* d_node_tri, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (first < 0 || last >= kNumBins || first > last)
    return fail(TRICC_EINVAL, "bin range %d..%d out of range", first, last);
  for (int b = first + 1; b <= last; ++b)
    if (g->tuning.bin_variant[b] != g->tuning.bin_variant[first])
      return fail(TRICC_EINVAL, "bins %d..%d do not share one kernel variant", first, last);
  return count_bins(g, first, last, d_node_tri, stream);
}

int tricc_count_finish(tricc_graph* g, const uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_total,
                       double* d_avg_cc, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if ((g->n > 0 && (!d_node_tri || !d_node_cc)) || !d_total || !d_avg_cc) return fail(TRICC_EINVAL, "null output");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = g->L;
  double* part_cc = g->at<double>(L.part_cc);
  unsigned long long* part_T = g->at<unsigned long long>(L.part_T);
  const unsigned long long* T = reinterpret_cast<const unsigned long long*>(d_node_tri);
  HIPCHK(launch_epilogue(g->n, T, g->at<int32_t>(L.deg), d_node_cc, part_cc, part_T, s));
  unsigned long long* check = reinterpret_cast<unsigned long long*>(g->ws + L.hdr + kHdrCheck * 4);
  HIPCHK(launch_finish(epilogue_blocks(g->n), g->n, part_cc, part_T, g->at<unsigned long long>(L.tot),
                       reinterpret_cast<unsigned long long*>(d_total), d_avg_cc, check + 1, s));
  HIPCHK(hipMemcpyAsync(check, d_total, sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
  return TRICC_OK;
}

int tricc_count_check(const tricc_graph* g, uint64_t* h_total, uint64_t* h_sum_T, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  unsigned long long v[2];
  int rc = sync_copy(v, g->ws + g->L.hdr + kHdrCheck * 4, sizeof(v), static_cast<hipStream_t>(stream));
  if (rc) return rc;
  if (h_total) *h_total = v[0];
  if (h_sum_T) *h_sum_T = v[1];
  return TRICC_OK;
}

int tricc_count(tricc_graph* g, uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_total, double* d_avg_cc,
                void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if ((g->n > 0 && (!d_node_tri || !d_node_cc)) || !d_total || !d_avg_cc)
    return fail(TRICC_EINVAL, "null output");
  int rc = tricc_count_begin(g, d_node_tri, stream);
  for (int b0 = 0; b0 < kNumBins && !rc;) {
    // adjacent bins with one variant run as one launch
    int b1 = b0;
    while (b1 + 1 < kNumBins && g->tuning.bin_variant[b1 + 1] == g->tuning.bin_variant[b0]) ++b1;
    rc = count_bins(g, b0, b1, d_node_tri, stream);
    b0 = b1 + 1;
  }
  if (!rc) rc = tricc_count_finish(g, d_node_tri, d_node_cc, d_total, d_avg_cc, stream);
  return rc;
}

int tricc_probe_copy(void* d_dst, const void* d_src, size_t bytes, void* stream) {
  if (bytes % 16 || reinterpret_cast<uintptr_t>(d_dst) % 16 || reinterpret_cast<uintptr_t>(d_src) % 16)
    return fail(TRICC_EINVAL, "probe copy needs 16-byte multiples and alignment");
  if (bytes && (!d_dst || !d_src)) return fail(TRICC_EINVAL, "null pointer");
  HIPCHK(launch_probe_copy(d_dst, d_src, bytes, static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

int tricc_gen_rmat(int32_t scale, int64_t m, double a, double b, double c, double d, double noise, uint64_t seed,
                   const int32_t* d_perm, int32_t* d_src, int32_t* d_dst, void* stream) {
  if (scale < 1 || scale > 30) return fail(TRICC_EINVAL, "R-MAT scale must be in [1, 30]");
  if (m < 0) return fail(TRICC_EINVAL, "negative edge count");
  const double abcd[4] = {a, b, c, d};
  double sum = 0.0;
  for (double w : abcd) {
    if (!std::isfinite(w) || w < 0.0) return fail(TRICC_EINVAL, "R-MAT weights must be finite and >= 0");
    sum += w;
  }
  if (!(sum > 0.0)) return fail(TRICC_EINVAL, "R-MAT weights sum to zero");
  if (!(noise >= 0.0 && noise <= 1.0)) return fail(TRICC_EINVAL, "R-MAT noise must be in [0, 1]");
  if (m > 0 && (!d_src || !d_dst)) return fail(TRICC_EINVAL, "null pointer");
  HIPCHK(launch_gen_rmat(m, scale, abcd, noise, seed, d_perm, d_src, d_dst, static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

}  // extern "C"

namespace {

// Draws the G(n, m) sampler runs: enough that fewer than m distinct values
// among them is far beyond the sampler's spread (about 10 standard deviations
// of the number of draws the m-th distinct value needs, or the coupon
// collector's tail when m > N/2).
int64_t er_draws(uint64_t N, int64_t m) {
  if (m <= 0) return 0;
  const double Nd = (double)N, f = (double)m / Nd;
  double K;
  if (2 * (uint64_t)m <= N) {
    const double e = -Nd * std::log1p(-f);
    const double var = Nd * (1.0 / (1.0 - f) - 1.0 + std::log1p(-f));
    K = e + 10.0 * std::sqrt(std::max(var, 0.0)) + 16.0;
  } else {
    K = Nd * (std::log(Nd) + 12.0);
  }
  return (int64_t)std::ceil(K) + 1024;
}

struct ErLayout {
  uint64_t P;
  int64_t K;
  size_t keys, idx, flag, pos, tmp, total;
};

int er_layout(int64_t n, int64_t m, ErLayout* L) {
  if (n < 0 || n > 0x7fffffffLL) return fail(TRICC_EINVAL, "G(n, m): n outside [0, 2^31 - 1]");
  const uint64_t N = n > 1 ? (uint64_t)n * (uint64_t)(n - 1) / 2 : 0;
  if (m < 0 || (uint64_t)m > N) return fail(TRICC_EINVAL, "G(n, m): m outside [0, n(n-1)/2]");
  if (m > (int64_t(1) << 30)) return fail(TRICC_EOVERFLOW, "G(n, m): m above 2^30");
  const int64_t K = er_draws(N, m);
  if (K >= (int64_t)0xFFFFFFFFLL) return fail(TRICC_EOVERFLOW, "G(n, m): too dense for the draw budget");
  uint64_t P = 1;
  while (P < 2 * (uint64_t)std::max<int64_t>(K, 1)) P <<= 1;
  size_t p = 0;
  auto take = [&](size_t bytes) { size_t at = p; p = align_up(p + std::max<size_t>(bytes, 1)); return at; };
  L->P = P;
  L->K = K;
  L->keys = take(sizeof(uint64_t) * P);
  L->idx = take(sizeof(uint32_t) * P);
  L->flag = take(sizeof(int32_t) * K);
  L->pos = take(sizeof(int64_t) * (K + 1));
  L->tmp = take(sizeof(int64_t) * scan_tmp_elems(K + 1));
  L->total = p;
  return TRICC_OK;
}

}  // namespace

extern "C" {

int tricc_gen_er_workspace_size(int64_t n, int64_t m, size_t* bytes) {
  if (!bytes) return fail(TRICC_EINVAL, "null bytes");
  ErLayout L;
  int rc = er_layout(n, m, &L);
  if (rc) return rc;
  *bytes = L.total;
  return TRICC_OK;
}

int tricc_gen_er(int64_t n, int64_t m, uint64_t seed, int32_t* d_src, int32_t* d_dst, void* d_ws, size_t ws_bytes,
                 void* stream) {
  ErLayout L;
  int rc = er_layout(n, m, &L);
  if (rc) return rc;
  if (m == 0) return TRICC_OK;
  if (!d_src || !d_dst) return fail(TRICC_EINVAL, "null output arrays");
  if (!d_ws || ws_bytes < L.total) return fail(TRICC_ENOMEM, "G(n, m) workspace %zu bytes, need %zu", ws_bytes, L.total);
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(TRICC_EINVAL, "workspace not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(d_ws);
  uint64_t* keys = reinterpret_cast<uint64_t*>(w + L.keys);
  uint32_t* idx = reinterpret_cast<uint32_t*>(w + L.idx);
  int32_t* flag = reinterpret_cast<int32_t*>(w + L.flag);
  int64_t* pos = reinterpret_cast<int64_t*>(w + L.pos);
  const uint64_t N = (uint64_t)n * (uint64_t)(n - 1) / 2;
  HIPCHK(launch_er_clear(L.P, keys, idx, s));
  HIPCHK(launch_er_insert(L.K, N, seed, L.P - 1, keys, idx, s));
  HIPCHK(launch_er_flag(L.K, N, seed, L.P - 1, keys, idx, flag, s));
  HIPCHK(launch_scan_i32(flag, L.K, pos, reinterpret_cast<int64_t*>(w + L.tmp), s));
  int64_t distinct = 0;
  if ((rc = sync_copy(&distinct, pos + L.K, sizeof(distinct), s))) return rc;
  if (distinct < m)
    return fail(TRICC_EOVERFLOW, "G(n, m): %lld distinct pairs in %lld draws, %lld needed", (long long)distinct,
                (long long)L.K, (long long)m);
  HIPCHK(launch_er_emit(L.K, n, N, seed, m, flag, pos, d_src, d_dst, s));
  return TRICC_OK;
}

int64_t tricc_gen_ba_edges(int64_t n, int32_t k) {
  if (k < 1 || k > 255 || n < k + 1 || n > 0x7fffffffLL) return -1;
  return (int64_t)k * (k + 1) / 2 + (n - k - 1) * (int64_t)k;
}

int tricc_gen_ba_workspace_size(int64_t n, int32_t k, size_t* bytes) {
  if (!bytes) return fail(TRICC_EINVAL, "null bytes");
  if (tricc_gen_ba_edges(n, k) < 0) return fail(TRICC_EINVAL, "Barabasi-Albert: need 1 <= k <= 255, k < n < 2^31");
  *bytes = align_up(sizeof(int32_t) * (size_t)n) + 256;
  return TRICC_OK;
}

int tricc_gen_ba(int64_t n, int32_t k, uint64_t seed, int32_t* d_src, int32_t* d_dst, void* d_ws, size_t ws_bytes,
                 void* stream) {
  const int64_t m = tricc_gen_ba_edges(n, k);
  if (m < 0) return fail(TRICC_EINVAL, "Barabasi-Albert: need 1 <= k <= 255, k < n < 2^31");
  if (m > (int64_t(1) << 30)) return fail(TRICC_EOVERFLOW, "Barabasi-Albert: more than 2^30 edges");
  if (!d_src || !d_dst) return fail(TRICC_EINVAL, "null output arrays");
  size_t need = 0;
  tricc_gen_ba_workspace_size(n, k, &need);
  if (!d_ws || ws_bytes < need) return fail(TRICC_ENOMEM, "Barabasi-Albert workspace %zu bytes, need %zu", ws_bytes, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(d_ws);
  int32_t* prog = reinterpret_cast<int32_t*>(w);
  int32_t* cnt = reinterpret_cast<int32_t*>(w + align_up(sizeof(int32_t) * (size_t)n));
  HIPCHK(launch_ba_init(m, k, (int32_t)n, d_src, d_dst, prog, cnt, s));
  int32_t c[2] = {1, 0};
  int rc;
  for (int pass = 0; c[0] > 0; ++pass) {
    if (pass >= (1 << 20)) return fail(TRICC_EHIP, "Barabasi-Albert: passes did not converge");
    HIPCHK(launch_ba_pass((int32_t)n, k, seed, d_src, d_dst, prog, cnt, s));
    if ((rc = sync_copy(c, cnt, sizeof(c), s))) return rc;
    if (c[1]) return fail(TRICC_EOVERFLOW, "Barabasi-Albert: an edge ran out of attempts");
  }
  return TRICC_OK;
}

int tricc_graph_arrays(const tricc_graph* g, const int64_t** d_off, const int32_t** d_deg, const int32_t** d_adj,
                       const int64_t** d_doff, const int32_t** d_dcol) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (d_off) *d_off = g->at<int64_t>(g->L.raw_off);
  if (d_deg) *d_deg = g->at<int32_t>(g->L.deg);
  if (d_adj) *d_adj = g->at<int32_t>(g->L.adj);
  if (d_doff) *d_doff = g->at<int64_t>(g->L.doff);
  if (d_dcol) *d_dcol = g->at<int32_t>(g->L.dcol);
  return TRICC_OK;
}

int tricc_graph_has_edges(const tricc_graph* g, int64_t q, const int32_t* d_u, const int32_t* d_v,
                          uint8_t* d_out, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (q < 0) return fail(TRICC_EINVAL, "negative query count");
  if (q == 0) return TRICC_OK;
  if (!d_u || !d_v || !d_out) return fail(TRICC_EINVAL, "null query or output array");
  const Layout& L = g->L;
  HIPCHK(launch_has_edges(q, d_u, d_v, g->n, g->at<int32_t>(L.rec), g->at<int32_t>(L.adj), d_out,
                          static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

int tricc_core_workspace_size(int32_t n, size_t* bytes) {
  if (n < 0 || !bytes) return fail(TRICC_EINVAL, "bad core workspace query");
  *bytes = 7 * align_up(sizeof(int32_t) * (size_t)std::max(n, 1)) + 256;
  return TRICC_OK;
}

}  // extern "C"

namespace {

// Levels per window of the core peeling: a scan of every node left opens a
// window [k, k + kCoreWindow], whose levels then scan the near list only.
constexpr int32_t kCoreWindow = 32;

// Peeling loop of the core decomposition; with d_order, every node's removal
// round as well (frontiers counted across levels).
int core_impl(const tricc_graph* g, int32_t k_stop, int32_t* d_core, int32_t* d_order, void* d_ws, size_t ws_bytes,
              int32_t* h_max_core, int32_t* h_rounds, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  const int32_t n = g->n;
  size_t need = 0;
  tricc_core_workspace_size(n, &need);
  if (n > 0 && (!d_core || !d_ws)) return fail(TRICC_EINVAL, "null core output or workspace");
  if (n > 0 && ws_bytes < need) return fail(TRICC_ENOMEM, "core workspace of %zu bytes, %zu needed", ws_bytes, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t maxc = 0, round = 0;
  if (n > 0) {
    char* w = static_cast<char*>(d_ws);
    const size_t slice = align_up(sizeof(int32_t) * (size_t)n);
    int32_t* cur = reinterpret_cast<int32_t*>(w);
    int32_t* F = reinterpret_cast<int32_t*>(w + slice);
    int32_t* G = reinterpret_cast<int32_t*>(w + 2 * slice);
    int32_t* A = reinterpret_cast<int32_t*>(w + 3 * slice);  // nodes left, listed by the last full scan
    int32_t* S = reinterpret_cast<int32_t*>(w + 4 * slice);
    int32_t* near[2] = {reinterpret_cast<int32_t*>(w + 5 * slice), reinterpret_cast<int32_t*>(w + 6 * slice)};
    int32_t* cnt = reinterpret_cast<int32_t*>(w + 7 * slice);
    const Layout& L = g->L;
    const int64_t* off = g->at<int64_t>(L.raw_off);
    const int32_t* deg = g->at<int32_t>(L.deg);
    const int32_t* adj = g->at<int32_t>(L.adj);
    HIPCHK(launch_core_init(n, deg, cur, d_core, s));
    int64_t left = n;
    int32_t k = 0;
    int rc;
    // full-scan candidates: all ids, until at most a quarter of the nodes
    // are left; from then on each full scan lists the survivors for the next
    const int32_t* cand = nullptr;
    int32_t ncand = n;
    // the window of levels [.., U] and its near list near[x] (length nx):
    // every node left with current degree <= U is on it
    int32_t U = -1, nx = 0, x = 0;
    while (left > 0 && (k_stop < 0 || k < k_stop)) {
      const bool full = k > U || nx == 0;
      const int y = x ^ 1;  // the scan lists this level's near nodes in near[y]
      int32_t c[8];
      if (full) {
        U = k + kCoreWindow;
        if (k_stop >= 0) U = std::min(U, k_stop - 1);  // no level at or above k_stop is peeled
        const bool listing = cand != nullptr || left <= n / 4;
        HIPCHK(launch_core_reset(cnt, 0, 6 + y, s));
        HIPCHK(launch_core_scan(ncand, cand, k, cur, d_core, F, listing ? S : nullptr, cnt, d_order, round, U, near[y],
                                cnt + 6 + y, s));
        if ((rc = sync_copy(c, cnt, sizeof(c), s))) return rc;
        if (listing) {
          std::swap(A, S);
          cand = A;
          ncand = c[3];
        }
      } else {
        HIPCHK(launch_core_reset(cnt, 0, 6 + y, s));
        HIPCHK(launch_core_scan(nx, near[x], k, cur, d_core, F, nullptr, cnt, d_order, round, U, near[y], cnt + 6 + y,
                                s));
        if ((rc = sync_copy(c, cnt, sizeof(c), s))) return rc;
      }
      x = y;
      nx = c[6 + x];
      if (c[0] == 0) {  // no node at this level: jump to the smallest current degree seen
        if (c[2] == 0x7fffffff) {
          if (full) break;  // no node left at all
          k = U + 1;        // none left in the window: every node left is above U
        } else {
          k = c[2];
        }
        continue;
      }
      int32_t nf = c[0];
      const int R = core_peel_batch();  // even: the frontier left ends in F
      while (nf > 0) {
        // R rounds per read-back; the ones after the level's last frontier
        // find an empty frontier and do nothing
        HIPCHK(launch_core_peel_batch(F, G, nf, k, off, deg, adj, cur, d_core, cnt, d_order, round, U, near[x],
                                      cnt + 6 + x, s));
        int32_t b[16 + 8];
        if ((rc = sync_copy(b, cnt, sizeof(int32_t) * (16 + R), s))) return rc;
        left -= nf;
        for (int i = 0; i + 1 < R; ++i) left -= b[16 + i];
        round += R;
        nf = b[16 + R - 1];
        c[6 + x] = b[6 + x];
      }
      nx = c[6 + x];
      maxc = k;
      ++k;
    }
    if (k_stop >= 0 && left > 0) {
      HIPCHK(launch_core_fill(n, k_stop, d_core, s));
      maxc = k_stop;
    }
    HIPCHK(hipStreamSynchronize(s));
  }
  if (h_max_core) *h_max_core = maxc;
  if (h_rounds) *h_rounds = round;
  return TRICC_OK;
}

}  // namespace

extern "C" {

int tricc_graph_core(const tricc_graph* g, int32_t k_stop, int32_t* d_core, void* d_ws, size_t ws_bytes,
                     int32_t* h_max_core, void* stream) {
  return core_impl(g, k_stop, d_core, nullptr, d_ws, ws_bytes, h_max_core, nullptr, stream);
}

int tricc_graph_degeneracy(const tricc_graph* g, int32_t* d_order, int32_t* d_core, void* d_ws, size_t ws_bytes,
                           int32_t* h_degeneracy, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (g->n > 0 && (!d_order || !d_core)) return fail(TRICC_EINVAL, "null order or core output");
  return core_impl(g, -1, d_core, d_order, d_ws, ws_bytes, h_degeneracy, nullptr, stream);
}

int tricc_graph_reorient(tricc_graph* g, const int32_t* d_key, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  g->stream = static_cast<hipStream_t>(stream);
  std::memset(g->info.bin_list_elems, 0, sizeof(g->info.bin_list_elems));
  g->info.list_elems = 0;
  return orient_impl(g, d_key);
}



int tricc_graph_count_k4(const tricc_graph* g, uint64_t* d_total, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (!d_total) return fail(TRICC_EINVAL, "null output");
  if (g->info.max_outdeg > kK4Cap)
    return fail(TRICC_EOVERFLOW, "4-clique counting takes out-degrees up to %d (this graph: %lld)", kK4Cap,
                (long long)g->info.max_outdeg);
  const Layout& L = g->L;
  HIPCHK(launch_count_k4(g->n, g->at<int64_t>(L.doff), g->at<int32_t>(L.dcol),
                         reinterpret_cast<unsigned long long*>(d_total), static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

int tricc_graph_count_k5(const tricc_graph* g, uint64_t* d_total, void* stream) {
  if (!g) return fail(TRICC_EINVAL, "null graph");
  if (!d_total) return fail(TRICC_EINVAL, "null output");
  if (g->info.max_outdeg > kK5Cap)
    return fail(TRICC_EOVERFLOW, "5-clique counting takes out-degrees up to %d (this graph: %lld)", kK5Cap,
                (long long)g->info.max_outdeg);
  const Layout& L = g->L;
  HIPCHK(launch_count_k5(g->n, g->at<int64_t>(L.doff), g->at<int32_t>(L.dcol),
                         reinterpret_cast<unsigned long long*>(d_total), static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

void tricc_graph_free(tricc_graph* g) { delete g; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Count without allocating: the graph workspace of a small graph lives in a
// file-scope device array (one copy per GPU, held until the process ends).
// Host code must not pass the array's name to a kernel (that is a host-side
// stand-in): its device address comes from hipGetSymbolAddress, once per
// device, and only that address is used.
namespace {

constexpr size_t kNoAllocBytes = TRICC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int scratch_for_current_device(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(TRICC_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % kAlign) return fail(TRICC_EHIP, "scratch symbol address unusable");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return TRICC_OK;
}

}  // namespace

extern "C" {

int tricc_count_noalloc(int32_t n, int64_t m_raw, const int32_t* d_src, const int32_t* d_dst, uint64_t* d_node_tri,
                        float* d_node_cc, uint64_t* d_total, double* d_avg_cc, void* stream) {
  g_err[0] = 0;
  if (n < 0 || m_raw < 0) return fail(TRICC_EINVAL, "negative size");
  if (n > TRICC_NOALLOC_MAX_NODES || m_raw > TRICC_NOALLOC_MAX_PAIRS)
    return fail(TRICC_EOVERFLOW, "tricc_count_noalloc takes n <= %d and m_raw <= %lld (got n = %d, m_raw = %lld)",
                TRICC_NOALLOC_MAX_NODES, (long long)TRICC_NOALLOC_MAX_PAIRS, n, (long long)m_raw);
  if (m_raw > 0 && (!d_src || !d_dst)) return fail(TRICC_EINVAL, "null edge arrays");
  if ((n > 0 && (!d_node_tri || !d_node_cc)) || !d_total || !d_avg_cc) return fail(TRICC_EINVAL, "null output");
  const Layout L = make_layout(n, m_raw);
  if (L.total > kNoAllocBytes)
    return fail(TRICC_EOVERFLOW, "graph needs %zu bytes of scratch, %zu available", L.total, kNoAllocBytes);
  char* ws = nullptr;
  int rc = scratch_for_current_device(&ws);
  if (rc) return rc;
  // the handle lives on this stack frame: no host or device allocation
  tricc_graph g;
  g.n = n;
  g.m_raw = m_raw;
  g.ws = ws;
  g.L = L;
  g.stream = static_cast<hipStream_t>(stream);
  tricc_default_tuning_impl(&g.tuning);
  std::memset(&g.info, 0, sizeof(g.info));
  if ((rc = build_impl(&g, d_src, d_dst))) return rc;
  return tricc_count(&g, d_node_tri, d_node_cc, d_total, d_avg_cc, stream);
}

}  // extern "C"

// ===========================================================================
// Batched graphs
// ===========================================================================
struct tricc_batch {
  int32_t G = 0;
  int64_t n_total = 0, m_total = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t* d_node_off = nullptr;
  int64_t* d_edge_off = nullptr;
  int32_t* d_queue = nullptr;
  int32_t* d_err = nullptr;
  int32_t* gsrc = nullptr;
  int32_t* gdst = nullptr;
  tricc_graph g;
  tricc_batch_tuning tuning{};
  unsigned grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  unsigned long long* T = nullptr;
  float* cc = nullptr;
  unsigned long long* graph_tri = nullptr;
  double* graph_avg = nullptr;
  unsigned long long* batch_tri = nullptr;
  int32_t* d_seg = nullptr;   // phase-2 segment bounds of the persistent kernel
  int64_t* d_thr = nullptr;   // first node of each segment
  std::vector<int64_t> h_node_off, h_edge_off;
  bool bound = false;
};

namespace {

struct BatchLayout {
  size_t hdr, node_off, edge_off, gsrc, gdst, graph_ws, total;
};

// Header: queue counters at byte 0 (2 + kPersistSegs int32), the error flag
// at 64, the segment bounds at 128 (2 (kPersistSegs + 1) int32), the segment
// thresholds at 256 (kPersistSegs + 1 int64).
constexpr size_t kBatchHdr = 512;

BatchLayout make_batch_layout(int64_t G, int64_t n_total, int64_t m_total) {
  BatchLayout L{};
  size_t p = 0;
  auto take = [&](size_t bytes) { size_t at = p; p = align_up(p + std::max<size_t>(bytes, 1)); return at; };
  L.hdr = take(kBatchHdr);
  L.node_off = take(sizeof(int64_t) * (G + 1));
  L.edge_off = take(sizeof(int64_t) * (G + 1));
  L.gsrc = take(sizeof(int32_t) * m_total);
  L.gdst = take(sizeof(int32_t) * m_total);
  L.graph_ws = p;
  L.total = p + make_layout(n_total, m_total).total;
  return L;
}

int check_batch_tuning(const tricc_batch_tuning* t) {
  if (t->persist_variant < 0 || t->persist_variant >= persist_variant_count())
    return fail(TRICC_EINVAL, "batch tuning: unknown persistent variant %d", t->persist_variant);
  if (t->wave_limit < 2 || t->wave_limit > persist_wave_cap(t->persist_variant))
    return fail(TRICC_EINVAL, "batch tuning: wave_limit %d outside [2, %d]", t->wave_limit,
                persist_wave_cap(t->persist_variant));
  if (t->merge_limit < 0 || t->merge_limit > t->wave_limit)
    return fail(TRICC_EINVAL, "batch tuning: merge_limit %d outside [0, wave_limit]", t->merge_limit);
  if (t->merge_limit > persist_merge_cap(t->persist_variant))
    return fail(TRICC_EINVAL, "batch tuning: merge_limit %d above %d for persistent variant %d", t->merge_limit,
                persist_merge_cap(t->persist_variant), t->persist_variant);
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > 64) return fail(TRICC_EINVAL, "batch tuning: blocks_per_cu");
  return TRICC_OK;
}

// Bins of the union graph: bin 0 = merge nodes (d+ <= merge_limit), bin 1
// = single-wave nodes (d+ <= wave_limit), bin 2 = block nodes (d+ <= the
// persistent block table's capacity): all three, and bin 5 (d+ > 4096,
// global fallback), run in the persistent kernel; bins 3 (up to 1024) and 4
// (up to 4096) run before it with the large-table kernel variants. The
// single-graph variants are set so that tricc_count also works on the union.
constexpr int kBatchVarBin3 = 15;  // 512 threads, cuckoo table for d+ <= 1024
constexpr int kBatchVarBin4 = 14;  // 1024 threads, cuckoo table for d+ <= 4096
// variants for bins 0..2 and 5 when tricc_count runs on the union graph
// (min_side 0: every edge counted from its tail)
constexpr int kBatchVarWave = 11;       // one wavefront per node, d+ <= 64
constexpr int kBatchVarBlock256 = 12;   // d+ <= 256
constexpr int kBatchVarBlock1024 = 13;  // d+ <= 1024
constexpr int kBatchVarGlobal = 8;
void batch_graph_tuning(const tricc_batch_tuning& bt, tricc_tuning* t) {
  const int32_t cb = persist_block_cap(bt.persist_variant);
  const int32_t lim[kNumBins - 1] = {bt.merge_limit, bt.wave_limit, cb, std::max(cb, 1024), 4096};
  const int32_t var[kNumBins] = {kBatchVarWave, kBatchVarWave, cb <= 256 ? kBatchVarBlock256 : kBatchVarBlock1024,
                                 kBatchVarBin3, kBatchVarBin4, kBatchVarGlobal};
  std::memcpy(t->bin_limit, lim, sizeof(lim));
  std::memcpy(t->bin_variant, var, sizeof(var));
  t->min_side = 0;
}

int batch_bin(tricc_batch* b) {
  batch_graph_tuning(b->tuning, &b->g.tuning);
  int rc = bin_nodes(&b->g);
  if (rc) return rc;
  // phase-2 segments: consecutive graphs with equal shares of the input pairs
  {
    const int32_t G = b->G;
    int64_t thr[kPersistSegs + 1];
    const int64_t E = G > 0 ? b->h_edge_off[G] : 0;
    int32_t gi = 0;
    thr[0] = 0;
    for (int x = 1; x < kPersistSegs; ++x) {
      const int64_t target = E * x / kPersistSegs;
      while (gi < G && b->h_edge_off[gi] < target) ++gi;
      thr[x] = G > 0 ? b->h_node_off[gi] : 0;
    }
    thr[kPersistSegs] = b->n_total;
    if ((rc = upload(b->d_thr, thr, sizeof(thr), b->g.stream))) return rc;
    const tricc_graph* g = &b->g;
    const int32_t* binlist = g->at<int32_t>(g->L.binlist);
    HIPCHK(launch_persist_segments(binlist + g->bin_off[1], (int32_t)(g->bin_off[2] - g->bin_off[1]),
                                   binlist + g->bin_off[0], (int32_t)(g->bin_off[1] - g->bin_off[0]), b->d_thr,
                                   b->d_seg, b->g.stream));
    HIPCHK(hipStreamSynchronize(b->g.stream));
  }
  int dev = 0, cus = 0, occ = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, persist_kernel(b->tuning.persist_variant), 256, 0));
  if (occ < 1) occ = 1;
  const int per = b->tuning.blocks_per_cu > 0 ? std::min(b->tuning.blocks_per_cu, occ) : occ;
  b->grid = (unsigned)std::max(1, cus * per);
  return TRICC_OK;
}

int batch_launch(tricc_batch* b, hipStream_t s) {
  tricc_graph* g = &b->g;
  const Layout& L = g->L;
  const int32_t* binlist = g->at<int32_t>(L.binlist);
  unsigned long long* tot = g->at<unsigned long long>(L.tot);
  HIPCHK(launch_batch_zero(b->T, b->n_total, tot, b->d_queue, s));
  // the heaviest nodes first, with the large LDS tables
  for (int bin = 4; bin >= 3; --bin) {
    BinLaunch bl{g->tuning.bin_variant[bin], binlist + g->bin_off[bin], (int32_t)(g->bin_off[bin + 1] - g->bin_off[bin])};
    HIPCHK(launch_count_bin(bl, g->at<int64_t>(L.doff), g->at<int32_t>(L.dcol), b->T, tot, s));
  }
  const int32_t nbk = (int32_t)(g->bin_off[3] - g->bin_off[2]);
  const int32_t ng = (int32_t)(g->bin_off[kNumBins] - g->bin_off[kNumBins - 1]);
  HIPCHK(launch_count_persist(b->tuning.persist_variant, b->grid, binlist + g->bin_off[kNumBins - 1], ng,
                              binlist + g->bin_off[2], nbk, binlist + g->bin_off[1], binlist + g->bin_off[0],
                              b->d_seg, b->d_queue, g->at<int64_t>(L.doff), g->at<int32_t>(L.dcol), b->T, tot, s));
  HIPCHK(launch_graph_epilogue(b->G, b->d_node_off, b->T, g->at<int32_t>(L.deg), b->cc, b->graph_tri, b->graph_avg,
                               tot, b->batch_tri, s));
  return TRICC_OK;
}

void batch_drop_plan(tricc_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

}  // namespace

extern "C" {

int tricc_batch_default_tuning(tricc_batch_tuning* out) {
  if (!out) return fail(TRICC_EINVAL, "null tuning");
  out->merge_limit = 16;
  out->wave_limit = 64;
  out->persist_variant = 2;
  out->blocks_per_cu = 0;
  return TRICC_OK;
}

int tricc_batch_workspace_size(int32_t num_graphs, int64_t total_nodes, int64_t total_pairs, size_t* bytes) {
  if (!bytes) return fail(TRICC_EINVAL, "null bytes");
  if (num_graphs < 0) return fail(TRICC_EINVAL, "negative graph count");
  if (total_nodes < 0 || total_nodes >= 0x7fffffff) return fail(TRICC_EINVAL, "total nodes out of range");
  if (total_pairs < 0) return fail(TRICC_EINVAL, "negative pair count");
  if (total_pairs > (int64_t(1) << 30)) return fail(TRICC_EOVERFLOW, "total pairs above 2^30");
  *bytes = make_batch_layout(num_graphs, total_nodes, total_pairs).total;
  return TRICC_OK;
}

int tricc_batch_build(int32_t num_graphs, const int64_t* h_node_off, const int64_t* h_edge_off, const int32_t* d_src,
                      const int32_t* d_dst, void* d_ws, size_t ws_bytes, const tricc_batch_tuning* tuning,
                      void* stream, tricc_batch** out) {
  g_err[0] = 0;
  if (!out) return fail(TRICC_EINVAL, "null out");
  *out = nullptr;
  if (num_graphs < 0 || (num_graphs > 0 && (!h_node_off || !h_edge_off)))
    return fail(TRICC_EINVAL, "bad graph count or offsets");
  const int64_t n_total = num_graphs ? h_node_off[num_graphs] : 0;
  const int64_t m_total = num_graphs ? h_edge_off[num_graphs] : 0;
  if (num_graphs && (h_node_off[0] != 0 || h_edge_off[0] != 0))
    return fail(TRICC_EINVAL, "offsets must start at 0");
  for (int32_t k = 0; k < num_graphs; ++k)
    if (h_node_off[k + 1] < h_node_off[k] || h_edge_off[k + 1] < h_edge_off[k])
      return fail(TRICC_EINVAL, "offsets must be non-decreasing");
  size_t need = 0;
  int rc = tricc_batch_workspace_size(num_graphs, n_total, m_total, &need);
  if (rc) return rc;
  if (m_total > 0 && (!d_src || !d_dst)) return fail(TRICC_EINVAL, "null edge arrays");
  if (!d_ws) return fail(TRICC_EINVAL, "null workspace");
  if (ws_bytes < need) return fail(TRICC_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(TRICC_EINVAL, "workspace not 256-byte aligned");
  tricc_batch_tuning bt;
  if (tuning) bt = *tuning; else tricc_batch_default_tuning(&bt);
  if ((rc = check_batch_tuning(&bt))) return rc;

  tricc_batch* b = new (std::nothrow) tricc_batch();
  if (!b) return fail(TRICC_ENOMEM, "host allocation failed");
  const BatchLayout BL = make_batch_layout(num_graphs, n_total, m_total);
  char* ws = static_cast<char*>(d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  b->G = num_graphs;
  b->n_total = n_total;
  b->m_total = m_total;
  b->ws = ws;
  b->ws_bytes = ws_bytes;
  b->d_queue = reinterpret_cast<int32_t*>(ws + BL.hdr);
  b->d_err = reinterpret_cast<int32_t*>(ws + BL.hdr + 64);
  b->d_seg = reinterpret_cast<int32_t*>(ws + BL.hdr + 128);
  b->d_thr = reinterpret_cast<int64_t*>(ws + BL.hdr + 256);
  b->d_node_off = reinterpret_cast<int64_t*>(ws + BL.node_off);
  b->d_edge_off = reinterpret_cast<int64_t*>(ws + BL.edge_off);
  b->gsrc = reinterpret_cast<int32_t*>(ws + BL.gsrc);
  b->gdst = reinterpret_cast<int32_t*>(ws + BL.gdst);
  b->tuning = bt;
  tricc_graph* g = &b->g;
  g->n = (int32_t)n_total;
  g->m_raw = m_total;
  g->ws = ws + BL.graph_ws;
  g->L = make_layout(n_total, m_total);
  g->stream = s;
  std::memset(&g->info, 0, sizeof(g->info));
  batch_graph_tuning(bt, &g->tuning);
  auto bail = [&](int code) { delete b; return code; };
  if (hipMemsetAsync(ws + BL.hdr, 0, kBatchHdr, s) != hipSuccess) return bail(fail(TRICC_EHIP, "memset failed"));
  if ((rc = upload(b->d_node_off, h_node_off, sizeof(int64_t) * (num_graphs + 1), s))) return bail(rc);
  if ((rc = upload(b->d_edge_off, h_edge_off, sizeof(int64_t) * (num_graphs + 1), s))) return bail(rc);
  b->h_node_off.assign(h_node_off, h_node_off + num_graphs + 1);
  b->h_edge_off.assign(h_edge_off, h_edge_off + num_graphs + 1);
  if (launch_batch_relabel(num_graphs, b->d_node_off, b->d_edge_off, d_src, d_dst, m_total, b->gsrc, b->gdst,
                           b->d_err, s) != hipSuccess)
    return bail(fail(TRICC_EHIP, "relabel launch failed"));
  int32_t err = 0;
  if ((rc = sync_copy(&err, b->d_err, sizeof(err), s))) return bail(rc);
  if (err) return bail(fail(TRICC_ERANGE, "a local node id is outside its graph's [0, n_g)"));
  if ((rc = build_impl(g, b->gsrc, b->gdst))) return bail(rc);
  if ((rc = batch_bin(b))) return bail(rc);
  *out = b;
  return TRICC_OK;
}

int tricc_batch_build_csr(int32_t num_graphs, const int64_t* h_node_off, int64_t nnz, const int64_t* d_rowptr,
                          const int32_t* d_col, int assume_simple_sorted_symmetric, void* d_ws, size_t ws_bytes,
                          const tricc_batch_tuning* tuning, void* stream, tricc_batch** out) {
  g_err[0] = 0;
  if (!out) return fail(TRICC_EINVAL, "null out");
  *out = nullptr;
  if (num_graphs < 0 || (num_graphs > 0 && !h_node_off)) return fail(TRICC_EINVAL, "bad graph count or offsets");
  if (nnz < 0) return fail(TRICC_EINVAL, "negative entry count");
  const int64_t n_total = num_graphs ? h_node_off[num_graphs] : 0;
  if (num_graphs && h_node_off[0] != 0) return fail(TRICC_EINVAL, "offsets must start at 0");
  for (int32_t k = 0; k < num_graphs; ++k)
    if (h_node_off[k + 1] < h_node_off[k]) return fail(TRICC_EINVAL, "offsets must be non-decreasing");
  size_t need = 0;
  int rc = tricc_batch_workspace_size(num_graphs, n_total, nnz, &need);
  if (rc) return rc;
  if (!d_rowptr || (nnz > 0 && !d_col)) return fail(TRICC_EINVAL, "null CSR arrays");
  if (!d_ws) return fail(TRICC_EINVAL, "null workspace");
  if (ws_bytes < need) return fail(TRICC_ENOMEM, "workspace %zu bytes, need %zu", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(TRICC_EINVAL, "workspace not 256-byte aligned");
  tricc_batch_tuning bt;
  if (tuning) bt = *tuning; else tricc_batch_default_tuning(&bt);
  if ((rc = check_batch_tuning(&bt))) return rc;

  tricc_batch* b = new (std::nothrow) tricc_batch();
  if (!b) return fail(TRICC_ENOMEM, "host allocation failed");
  const BatchLayout BL = make_batch_layout(num_graphs, n_total, nnz);
  char* ws = static_cast<char*>(d_ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  b->G = num_graphs;
  b->n_total = n_total;
  b->m_total = nnz;
  b->ws = ws;
  b->ws_bytes = ws_bytes;
  b->d_queue = reinterpret_cast<int32_t*>(ws + BL.hdr);
  b->d_err = reinterpret_cast<int32_t*>(ws + BL.hdr + 64);
  b->d_seg = reinterpret_cast<int32_t*>(ws + BL.hdr + 128);
  b->d_thr = reinterpret_cast<int64_t*>(ws + BL.hdr + 256);
  b->d_node_off = reinterpret_cast<int64_t*>(ws + BL.node_off);
  b->d_edge_off = reinterpret_cast<int64_t*>(ws + BL.edge_off);
  b->gsrc = reinterpret_cast<int32_t*>(ws + BL.gsrc);
  b->gdst = reinterpret_cast<int32_t*>(ws + BL.gdst);
  b->tuning = bt;
  tricc_graph* g = &b->g;
  g->n = (int32_t)n_total;
  g->m_raw = nnz;
  g->ws = ws + BL.graph_ws;
  g->L = make_layout(n_total, nnz);
  g->stream = s;
  std::memset(&g->info, 0, sizeof(g->info));
  batch_graph_tuning(bt, &g->tuning);
  auto bail = [&](int code) { delete b; return code; };
  if (hipMemsetAsync(ws + BL.hdr, 0, kBatchHdr, s) != hipSuccess) return bail(fail(TRICC_EHIP, "memset failed"));
  if ((rc = upload(b->d_node_off, h_node_off, sizeof(int64_t) * (num_graphs + 1), s))) return bail(rc);
  // the graphs' entry ranges, rowptr at the node boundaries; the row offsets
  // themselves are checked by the CSR build
  int64_t last = 0;
  if (num_graphs > 0) {
    if (launch_gather_offsets(d_rowptr, b->d_node_off, num_graphs + 1, b->d_edge_off, s) != hipSuccess)
      return bail(fail(TRICC_EHIP, "offset gather failed"));
    if ((rc = sync_copy(&last, b->d_edge_off + num_graphs, sizeof(last), s))) return bail(rc);
    if (last != nnz) return bail(fail(TRICC_EINVAL, "rowptr[total nodes] = %lld, expected nnz = %lld",
                                      (long long)last, (long long)nnz));
  }
  b->h_node_off.assign(h_node_off, h_node_off + num_graphs + 1);
  b->h_edge_off.assign(num_graphs + 1, 0);
  if (num_graphs > 0 && (rc = sync_copy(b->h_edge_off.data(), b->d_edge_off, sizeof(int64_t) * (num_graphs + 1), s)))
    return bail(rc);
  if (launch_batch_relabel(num_graphs, b->d_node_off, b->d_edge_off, nullptr, d_col, nnz, nullptr, b->gdst, b->d_err,
                           s) != hipSuccess)
    return bail(fail(TRICC_EHIP, "relabel launch failed"));
  int32_t err = 0;
  if ((rc = sync_copy(&err, b->d_err, sizeof(err), s))) return bail(rc);
  if (err) return bail(fail(TRICC_ERANGE, "a local node id is outside its graph's [0, n_g)"));
  if ((rc = csr_build(g, nnz, d_rowptr, b->gdst, assume_simple_sorted_symmetric))) return bail(rc);
  if ((rc = batch_bin(b))) return bail(rc);
  *out = b;
  return TRICC_OK;
}

int tricc_batch_plan(tricc_batch* b, uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_graph_tri, double* d_graph_avg,
                     uint64_t* d_batch_tri, void* stream) {
  if (!b) return fail(TRICC_EINVAL, "null batch");
  if ((b->n_total > 0 && (!d_node_tri || !d_node_cc)) || (b->G > 0 && (!d_graph_tri || !d_graph_avg)))
    return fail(TRICC_EINVAL, "null output");
  batch_drop_plan(b);
  b->T = reinterpret_cast<unsigned long long*>(d_node_tri);
  b->cc = d_node_cc;
  b->graph_tri = reinterpret_cast<unsigned long long*>(d_graph_tri);
  b->graph_avg = d_graph_avg;
  b->batch_tri = reinterpret_cast<unsigned long long*>(d_batch_tri);
  b->bound = true;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(hipStreamSynchronize(s));
  hipStream_t cs;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = TRICC_OK;
  if (e == hipSuccess) {
    rc = batch_launch(b, cs);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (rc == TRICC_OK && e2 != hipSuccess) rc = fail(TRICC_EHIP, "end capture: %s", hipGetErrorString(e2));
    if (rc == TRICC_OK) {
      b->graph = graph;
      e2 = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
      if (e2 != hipSuccess) rc = fail(TRICC_EHIP, "graph instantiate: %s", hipGetErrorString(e2));
    } else if (graph) {
      (void)hipGraphDestroy(graph);
    }
  } else {
    rc = fail(TRICC_EHIP, "begin capture: %s", hipGetErrorString(e));
  }
  (void)hipStreamDestroy(cs);
  if (rc) batch_drop_plan(b);
  return rc;
}

int tricc_batch_bind(tricc_batch* b, uint64_t* d_node_tri, float* d_node_cc, uint64_t* d_graph_tri,
                     double* d_graph_avg, uint64_t* d_batch_tri) {
  if (!b) return fail(TRICC_EINVAL, "null batch");
  if ((b->n_total > 0 && (!d_node_tri || !d_node_cc)) || (b->G > 0 && (!d_graph_tri || !d_graph_avg)))
    return fail(TRICC_EINVAL, "null output");
  batch_drop_plan(b);
  b->T = reinterpret_cast<unsigned long long*>(d_node_tri);
  b->cc = d_node_cc;
  b->graph_tri = reinterpret_cast<unsigned long long*>(d_graph_tri);
  b->graph_avg = d_graph_avg;
  b->batch_tri = reinterpret_cast<unsigned long long*>(d_batch_tri);
  b->bound = true;
  return TRICC_OK;
}

int tricc_batch_run(tricc_batch* b, void* stream) {
  if (!b) return fail(TRICC_EINVAL, "null batch");
  if (!b->exec) return fail(TRICC_EINVAL, "batch not planned");
  HIPCHK(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
  return TRICC_OK;
}

int tricc_batch_run_eager(tricc_batch* b, void* stream) {
  if (!b) return fail(TRICC_EINVAL, "null batch");
  if (!b->bound) return fail(TRICC_EINVAL, "batch outputs not bound (plan first)");
  return batch_launch(b, static_cast<hipStream_t>(stream));
}

int tricc_batch_retune(tricc_batch* b, const tricc_batch_tuning* tuning, void* stream) {
  if (!b || !tuning) return fail(TRICC_EINVAL, "null argument");
  int rc = check_batch_tuning(tuning);
  if (rc) return rc;
  batch_drop_plan(b);
  b->tuning = *tuning;
  b->g.stream = static_cast<hipStream_t>(stream);
  return batch_bin(b);
}

int tricc_batch_info_get(const tricc_batch* b, tricc_batch_info* out) {
  if (!b || !out) return fail(TRICC_EINVAL, "null argument");
  const tricc_graph& g = b->g;
  out->num_graphs = b->G;
  out->total_nodes = b->n_total;
  out->total_pairs = b->m_total;
  out->m = g.info.m;
  out->max_outdeg = g.info.max_outdeg;
  out->merge_nodes = g.bin_off[1] - g.bin_off[0];
  out->wave_nodes = g.bin_off[2] - g.bin_off[1];
  out->block_nodes = g.bin_off[3] - g.bin_off[2];
  out->hub_nodes = g.bin_off[kNumBins] - g.bin_off[3];  // large-table bins and the fallback
  out->grid = (int32_t)b->grid;
  out->planned = b->exec != nullptr;
  return TRICC_OK;
}

const tricc_graph* tricc_batch_graph(const tricc_batch* b) { return b ? &b->g : nullptr; }

void tricc_batch_free(tricc_batch* b) {
  if (!b) return;
  batch_drop_plan(b);
  delete b;
}

}  // extern "C"

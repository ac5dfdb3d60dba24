// Query server: induced-subgraph triangle counts and average clustering
// coefficients over a graph resident on the device, with memory-based
// admission and continuous batching.
//
// Each of `slots` worker threads owns a HIP stream and an equal slice of the
// caller's device workspace. A worker takes every waiting query that fits
// its slice (in arrival order, up to max_batch_queries), extracts their
// induced subgraphs on the device, builds them as one batch and counts them
// with the persistent kernel; queries that arrive meanwhile wait for the
// next free worker. Workers run concurrently, so their device work
// overlaps. A query's result depends only on the query: the per-graph
// epilogue sums in a fixed order, so it is bit-identical alone and in any
// mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/tricc.h"
#include "kernels.h"

namespace tricc {
hipError_t launch_serve_clear(int2* tab, int64_t total, hipStream_t s);
hipError_t launch_serve_insert(int32_t Q, const int64_t* qoff, const int32_t* nodes, int64_t N, const int64_t* toff,
                               int2* tab, int32_t n, const int32_t* deg, int32_t* nchunks, int32_t* qidx, int32_t* err,
                               hipStream_t s);
hipError_t launch_serve_items(int64_t N, const int64_t* coff, int32_t* item, hipStream_t s);
hipError_t launch_serve_pairs(int pass, int32_t Q, const int64_t* qoff, const int32_t* nodes, const int64_t* coff,
                              int64_t C, const int32_t* item, const int32_t* qidx, const int64_t* toff, const int2* tab,
                              const int64_t* off, const int32_t* deg, const int32_t* adj, int32_t* cnt,
                              const int64_t* pos, int32_t* psrc, int32_t* pdst, hipStream_t s);
hipError_t launch_serve_query_pairs(int32_t Q, const int64_t* qoff, const int64_t* coff, const int64_t* pos,
                                    int64_t* qpairs, hipStream_t s);
}  // namespace tricc

using namespace tricc;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int32_t kChunk = 2048;  // neighbours per extraction work item (serve_kernels.hip)

inline int64_t pow2_at_least(int64_t x) {
  int64_t p = 2;
  while (p < x) p <<= 1;
  return p;
}

// Device bytes a batch needs in a slot (extraction buffers + batch build),
// from an upper bound on its pairs. G queries, N nodes, D = sum of resident
// degrees of the nodes, M = bound on emitted pairs, T = table slots.
struct SlotLayout {
  size_t nodes, qoff, toff, tab, nchunks, qidx, coff, item, scan, cnt, pos, psrc, pdst, qpairs, err, T, cc, gtri,
      gavg, batch, total;
};

SlotLayout slot_layout(int64_t G, int64_t N, int64_t D, int64_t M, int64_t Tslots) {
  SlotLayout L{};
  size_t p = 0;
  auto take = [&](size_t bytes) { size_t at = p; p = align_up(p + std::max<size_t>(bytes, 1)); return at; };
  const int64_t C = N + D / kChunk + 1;  // chunks: sum over nodes of ceil(d / kChunk)
  L.nodes = take(4 * N);
  L.qoff = take(8 * (G + 1));
  L.toff = take(8 * (G + 1));
  L.tab = take(8 * Tslots);
  L.nchunks = take(4 * N);
  L.qidx = take(4 * N);  // query of each item
  L.coff = take(8 * (N + 1));
  L.item = take(4 * C);  // item of each chunk
  L.scan = take(8 * (std::max(N, C) / 4096 + 4));
  L.cnt = take(4 * C);
  L.pos = take(8 * (C + 1));
  L.psrc = take(4 * M);
  L.pdst = take(4 * M);
  L.qpairs = take(8 * (G + 1));
  L.err = take(64);
  L.T = take(8 * N);
  L.cc = take(4 * N);
  L.gtri = take(8 * G);
  L.gavg = take(8 * G);
  L.batch = p;
  size_t bws = 0;
  tricc_batch_workspace_size((int32_t)G, N, M, &bws);
  L.total = p + bws;
  return L;
}

struct Query {
  uint64_t qid;
  std::vector<int32_t> nodes;
  double t_arrival;
  int64_t deg_sum;  // sum of resident degrees of the nodes
  int64_t pairs_bound;
  int64_t tslots;
  size_t cost;  // device bytes of this query alone
};

int64_t pairs_bound(int64_t k, int64_t deg_sum) {
  const int64_t full = k * (k - 1) / 2;
  return std::min(full, deg_sum / 2 + 1);
}

thread_local char s_err[512] = "";

int sfail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(s_err, sizeof(s_err), fmt, ap);
  va_end(ap);
  return status;
}

}  // namespace

struct tricc_server {
  // resident graph (device)
  int32_t n = 0;
  int device = 0;
  const int64_t* off = nullptr;
  const int32_t* deg = nullptr;
  const int32_t* adj = nullptr;
  std::vector<int32_t> h_deg;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t slot_bytes = 0;
  int32_t nslots = 0;
  int32_t max_batch = 0;
  // state
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Query> waiting;
  std::vector<tricc_result> done;
  size_t outstanding = 0;  // bytes of admitted queries not yet completed
  int64_t in_flight = 0;   // admitted, not completed
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<int32_t> stamp;  // host-side id check
  int64_t stamp_epoch = 0;
  std::chrono::steady_clock::time_point t0;
  tricc_batch_tuning tuning{};
  int first_error = TRICC_OK;
  char first_error_text[512] = "";
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

#define SCHK(expr)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return sfail(TRICC_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// Runs one batch on a slot; fills results. Returns a TRICC status.
int run_batch(tricc_server* S, char* ws, hipStream_t st, std::vector<Query>& B, std::vector<tricc_result>& out,
              const tricc_batch_tuning& bt) {
  const int32_t G = (int32_t)B.size();
  int64_t N = 0, D = 0, M = 0, Tsl = 0;
  std::vector<int64_t> qoff(G + 1, 0), toff(G + 1, 0);
  for (int32_t q = 0; q < G; ++q) {
    N += (int64_t)B[q].nodes.size();
    D += B[q].deg_sum;
    M += B[q].pairs_bound;
    Tsl += B[q].tslots;
    qoff[q + 1] = N;
    toff[q + 1] = Tsl;
  }
  const SlotLayout L = slot_layout(G, N, D, M, Tsl);
  if (L.total > S->slot_bytes) return sfail(TRICC_ENOMEM, "batch needs %zu bytes, slot has %zu", L.total, S->slot_bytes);
  auto at = [&](size_t o) { return ws + o; };
  int32_t* nodes = reinterpret_cast<int32_t*>(at(L.nodes));
  int64_t* d_qoff = reinterpret_cast<int64_t*>(at(L.qoff));
  int64_t* d_toff = reinterpret_cast<int64_t*>(at(L.toff));
  int2* tab = reinterpret_cast<int2*>(at(L.tab));
  int32_t* nchunks = reinterpret_cast<int32_t*>(at(L.nchunks));
  int32_t* qidx = reinterpret_cast<int32_t*>(at(L.qidx));
  int64_t* coff = reinterpret_cast<int64_t*>(at(L.coff));
  int32_t* item = reinterpret_cast<int32_t*>(at(L.item));
  int64_t* scan = reinterpret_cast<int64_t*>(at(L.scan));
  int32_t* cnt = reinterpret_cast<int32_t*>(at(L.cnt));
  int64_t* pos = reinterpret_cast<int64_t*>(at(L.pos));
  int32_t* psrc = reinterpret_cast<int32_t*>(at(L.psrc));
  int32_t* pdst = reinterpret_cast<int32_t*>(at(L.pdst));
  int64_t* qpairs = reinterpret_cast<int64_t*>(at(L.qpairs));
  int32_t* err = reinterpret_cast<int32_t*>(at(L.err));
  uint64_t* T = reinterpret_cast<uint64_t*>(at(L.T));
  float* cc = reinterpret_cast<float*>(at(L.cc));
  uint64_t* gtri = reinterpret_cast<uint64_t*>(at(L.gtri));
  double* gavg = reinterpret_cast<double*>(at(L.gavg));

  // host staging of the node lists (copied synchronously from pageable memory)
  std::vector<int32_t> flat((size_t)N);
  for (int32_t q = 0; q < G; ++q) std::copy(B[q].nodes.begin(), B[q].nodes.end(), flat.begin() + qoff[q]);
  SCHK(hipMemcpyAsync(nodes, flat.data(), 4 * (size_t)N, hipMemcpyHostToDevice, st));
  SCHK(hipMemcpyAsync(d_qoff, qoff.data(), 8 * (size_t)(G + 1), hipMemcpyHostToDevice, st));
  SCHK(hipMemcpyAsync(d_toff, toff.data(), 8 * (size_t)(G + 1), hipMemcpyHostToDevice, st));
  SCHK(hipMemsetAsync(err, 0, 64, st));
  SCHK(launch_serve_clear(tab, Tsl, st));
  SCHK(launch_serve_insert(G, d_qoff, nodes, N, d_toff, tab, S->n, S->deg, nchunks, qidx, err, st));
  SCHK(launch_scan_i32(nchunks, N, coff, scan, st));
  int64_t C = 0;
  int32_t herr = 0;
  SCHK(hipMemcpyAsync(&C, coff + N, 8, hipMemcpyDeviceToHost, st));
  SCHK(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
  SCHK(hipStreamSynchronize(st));
  if (herr) return sfail(TRICC_EINVAL, "query node ids invalid on the device (flag %d)", herr);
  if (C > N + D / kChunk + 1) return sfail(TRICC_EOVERFLOW, "chunk bound exceeded");
  SCHK(launch_serve_items(N, coff, item, st));
  SCHK(launch_serve_pairs(0, G, d_qoff, nodes, coff, C, item, qidx, d_toff, tab, S->off, S->deg, S->adj, cnt, nullptr,
                          nullptr, nullptr, st));
  SCHK(launch_scan_i32(cnt, C, pos, scan, st));
  SCHK(launch_serve_query_pairs(G, d_qoff, coff, pos, qpairs, st));
  std::vector<int64_t> hq(G + 1);
  SCHK(hipMemcpyAsync(hq.data(), qpairs, 8 * (size_t)(G + 1), hipMemcpyDeviceToHost, st));
  SCHK(hipStreamSynchronize(st));
  if (hq[G] > M) return sfail(TRICC_EOVERFLOW, "pair bound exceeded");
  SCHK(launch_serve_pairs(1, G, d_qoff, nodes, coff, C, item, qidx, d_toff, tab, S->off, S->deg, S->adj, cnt, pos,
                          psrc, pdst, st));
  tricc_batch* b = nullptr;
  int rc = tricc_batch_build(G, qoff.data(), hq.data(), psrc, pdst, at(L.batch), S->slot_bytes - L.batch, &bt, st, &b);
  if (rc) return rc;
  rc = tricc_batch_bind(b, T, cc, gtri, gavg, nullptr);
  if (!rc) rc = tricc_batch_run_eager(b, st);
  std::vector<uint64_t> htri(G);
  std::vector<double> havg(G);
  if (!rc && G > 0) {
    if (hipMemcpyAsync(htri.data(), gtri, 8 * (size_t)G, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(havg.data(), gavg, 8 * (size_t)G, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = sfail(TRICC_EHIP, "result copy failed");
  }
  tricc_batch_free(b);
  if (rc) return rc;
  const double t_done = S->now();
  for (int32_t q = 0; q < G; ++q) {
    tricc_result r{};
    r.qid = B[q].qid;
    r.k = (int64_t)B[q].nodes.size();
    r.triangles = htri[q];
    r.avg_cc = havg[q];
    r.m = hq[q + 1] - hq[q];
    r.t_arrival = B[q].t_arrival;
    r.t_done = t_done;
    r.batch_size = G;
    r.status = TRICC_OK;
    out.push_back(r);
  }
  return TRICC_OK;
}

void worker_main(tricc_server* S, int slot) {
  if (hipSetDevice(S->device) != hipSuccess) return;
  hipStream_t st;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  char* ws = S->ws + (size_t)slot * S->slot_bytes;
  while (true) {
    std::vector<Query> B;
    tricc_batch_tuning bt;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->waiting.empty(); });
      if (S->waiting.empty() && S->stop) break;
      bt = S->tuning;
      // continuous batching: everything waiting that fits this slot, in order
      int64_t G = 0, N = 0, D = 0, M = 0, Tsl = 0;
      while (!S->waiting.empty() && G < S->max_batch) {
        const Query& q = S->waiting.front();
        const SlotLayout L = slot_layout(G + 1, N + (int64_t)q.nodes.size(), D + q.deg_sum, M + q.pairs_bound,
                                         Tsl + q.tslots);
        if (L.total > S->slot_bytes && G > 0) break;
        G += 1;
        N += (int64_t)q.nodes.size();
        D += q.deg_sum;
        M += q.pairs_bound;
        Tsl += q.tslots;
        B.push_back(std::move(S->waiting.front()));
        S->waiting.pop_front();
      }
    }
    const double t_start = S->now();
    std::vector<tricc_result> res;
    const int rc = run_batch(S, ws, st, B, res, bt);
    size_t freed = 0;
    for (const Query& q : B) freed += q.cost;
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc) {
      if (S->first_error == TRICC_OK) {
        S->first_error = rc;
        std::snprintf(S->first_error_text, sizeof(S->first_error_text), "%s", s_err);
      }
      for (const Query& q : B) {
        tricc_result r{};
        r.qid = q.qid;
        r.k = (int64_t)q.nodes.size();
        r.t_arrival = q.t_arrival;
        r.t_done = S->now();
        r.batch_size = (int32_t)B.size();
        r.status = rc;
        res.push_back(r);
      }
    }
    for (tricc_result& r : res) {
      r.t_start = t_start;
      S->done.push_back(r);
    }
    S->outstanding -= freed;
    S->in_flight -= (int64_t)B.size();
    S->cv_done.notify_all();
  }
  (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

const char* tricc_server_last_error(void) { return s_err; }

int tricc_server_create(const tricc_graph* resident, void* d_ws, size_t ws_bytes, int32_t slots,
                        int32_t max_batch_queries, tricc_server** out) {
  if (!out) return sfail(TRICC_EINVAL, "null out");
  *out = nullptr;
  if (!resident || !d_ws) return sfail(TRICC_EINVAL, "null resident graph or workspace");
  if (slots < 1 || slots > 16) return sfail(TRICC_EINVAL, "slots must be in [1, 16]");
  if (max_batch_queries < 1) return sfail(TRICC_EINVAL, "max_batch_queries must be >= 1");
  if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return sfail(TRICC_EINVAL, "workspace not 256-byte aligned");
  tricc_graph_info info;
  if (tricc_graph_info_get(resident, &info)) return sfail(TRICC_EINVAL, "bad resident graph");
  const int64_t* off = nullptr;
  const int32_t* deg = nullptr;
  const int32_t* adj = nullptr;
  tricc_graph_arrays(resident, &off, &deg, &adj, nullptr, nullptr);
  tricc_server* S = new (std::nothrow) tricc_server();
  if (!S) return sfail(TRICC_ENOMEM, "host allocation failed");
  S->n = info.n;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return sfail(TRICC_EHIP, "no current device");
  }
  S->off = off;
  S->deg = deg;
  S->adj = adj;
  S->h_deg.resize(info.n);
  if (info.n > 0 && hipMemcpy(S->h_deg.data(), deg, 4 * (size_t)info.n, hipMemcpyDeviceToHost) != hipSuccess) {
    delete S;
    return sfail(TRICC_EHIP, "degree copy failed");
  }
  S->ws = static_cast<char*>(d_ws);
  S->ws_bytes = ws_bytes;
  S->slot_bytes = ws_bytes / (size_t)slots / kAlign * kAlign;
  S->nslots = slots;
  S->max_batch = max_batch_queries;
  S->stamp.assign(info.n, -1);
  tricc_batch_default_tuning(&S->tuning);
  S->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < slots; ++i) S->workers.emplace_back(worker_main, S, i);
  *out = S;
  return TRICC_OK;
}

int tricc_server_set_tuning(tricc_server* s, const tricc_batch_tuning* tuning) {
  if (!s || !tuning) return sfail(TRICC_EINVAL, "null argument");
  const int pv = tuning->persist_variant;
  if (pv < 0 || pv >= tricc::persist_variant_count() || tuning->merge_limit < 0 ||
      tuning->wave_limit < tuning->merge_limit || tuning->wave_limit < 2 ||
      tuning->wave_limit > tricc::persist_wave_cap(pv) || tuning->merge_limit > tricc::persist_merge_cap(pv) ||
      tuning->blocks_per_cu < 0 || tuning->blocks_per_cu > 64)
    return sfail(TRICC_EINVAL, "bad batch tuning");
  std::lock_guard<std::mutex> lk(s->mu);
  s->tuning = *tuning;
  return TRICC_OK;
}

double tricc_server_now(const tricc_server* s) { return s ? s->now() : 0.0; }

int tricc_server_submit(tricc_server* s, uint64_t qid, const int32_t* h_nodes, int64_t k, double t_arrival) {
  if (!s) return sfail(TRICC_EINVAL, "null server");
  if (k < 0 || (k > 0 && !h_nodes)) return sfail(TRICC_EINVAL, "bad node list");
  if (k >= 0x7fffffff) return sfail(TRICC_EOVERFLOW, "query too large");
  Query q;
  q.qid = qid;
  q.t_arrival = t_arrival;
  q.nodes.assign(h_nodes, h_nodes + k);
  int64_t ds = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t epoch = ++s->stamp_epoch;
    for (int64_t i = 0; i < k; ++i) {
      const int32_t v = h_nodes[i];
      if (v < 0 || v >= s->n) return sfail(TRICC_ERANGE, "node id %d outside [0, %d)", v, s->n);
      if (s->stamp[v] == (int32_t)epoch) return sfail(TRICC_EINVAL, "node %d repeated in the query", v);
      s->stamp[v] = (int32_t)epoch;
      ds += s->h_deg[v];
    }
  }
  q.deg_sum = ds;
  q.pairs_bound = pairs_bound(k, ds);
  q.tslots = pow2_at_least(2 * k);
  q.cost = slot_layout(1, k, ds, q.pairs_bound, q.tslots).total;
  if (q.cost > s->slot_bytes)
    return sfail(TRICC_ENOMEM, "query needs %zu bytes, a slot has %zu", q.cost, s->slot_bytes);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->outstanding + q.cost > s->ws_bytes) return sfail(TRICC_EBUSY, "admission refused: memory budget in use");
  s->outstanding += q.cost;
  s->in_flight += 1;
  s->waiting.push_back(std::move(q));
  s->cv_work.notify_one();
  return TRICC_OK;
}

int tricc_server_poll(tricc_server* s, tricc_result* out, int32_t cap, int32_t* n_out) {
  if (!s || !n_out || (cap > 0 && !out)) return sfail(TRICC_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  const int32_t n = (int32_t)std::min<size_t>((size_t)cap, s->done.size());
  for (int32_t i = 0; i < n; ++i) out[i] = s->done[i];
  s->done.erase(s->done.begin(), s->done.begin() + n);
  *n_out = n;
  return TRICC_OK;
}

int tricc_server_drain(tricc_server* s) {
  if (!s) return sfail(TRICC_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->in_flight == 0; });
  if (s->first_error != TRICC_OK) {
    std::snprintf(s_err, sizeof(s_err), "%s", s->first_error_text);
    return s->first_error;
  }
  return TRICC_OK;
}

int tricc_server_stats(const tricc_server* s, int64_t* waiting, int64_t* in_flight, size_t* outstanding_bytes) {
  if (!s) return sfail(TRICC_EINVAL, "null server");
  tricc_server* m = const_cast<tricc_server*>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  if (waiting) *waiting = (int64_t)m->waiting.size();
  if (in_flight) *in_flight = m->in_flight;
  if (outstanding_bytes) *outstanding_bytes = m->outstanding;
  return TRICC_OK;
}

size_t tricc_server_query_bytes(const tricc_server* s, const int32_t* h_nodes, int64_t k) {
  if (!s || k < 0 || (k > 0 && !h_nodes)) return 0;
  int64_t ds = 0;
  for (int64_t i = 0; i < k; ++i)
    if (h_nodes[i] >= 0 && h_nodes[i] < s->n) ds += s->h_deg[h_nodes[i]];
  return slot_layout(1, k, ds, pairs_bound(k, ds), pow2_at_least(2 * k)).total;
}

void tricc_server_free(tricc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (std::thread& t : s->workers) t.join();
  delete s;
}

}  // extern "C"

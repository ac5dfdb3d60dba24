/*
 * CPU oracle for exact triangle counting, clustering coefficients,
 * edge-existence tests, core numbers, 4-clique counts and the R-MAT,
 * G(n, m) and Barabasi-Albert edge generators.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do. It shares no code, header or constant with the GPU path.
 *
 * What it computes (the paper lists "node clustering coefficient" and
 * "triangle counting" among SNAP's triadic-closure methods, in the table of
 * graph manipulation and analytics methods of Section 4; it states no
 * formula, so the plain graph-theoretic definitions are written out):
 *
 *   E     = { {u,v} : (u,v) or (v,u) is an input pair, u != v }   (undirected
 *           simple graph, Section 3.1: undirected edges, no explicit ids)
 *   N(v)  = sorted neighbours of v, d(v) = |N(v)|   (Section 5.1: every node
 *           keeps a sorted vector of adjacent nodes)
 *   T(v)  = number of pairs {u,w} in N(v) with {u,w} in E
 *   T     = number of node triples that are pairwise adjacent = sum T(v) / 3
 *   CC(v) = 2 T(v) / (d(v)(d(v)-1)) for d(v) >= 2, else 0      (FP64)
 *   avg   = (1/n) * sum over all n ids of CC(v)                 (FP64)
 *
 * Counting is the plain node iterator: every triangle is met once at its
 * lowest-ranked vertex v, through a neighbour u ranked above v and a
 * neighbour w of u ranked above u that is marked as a neighbour of v.
 * The rank is either the node id (order_mode 0) or the pair (d(v), v)
 * (order_mode 1); both must give identical results.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC tricc_oracle.c -o liboracle.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static int cmp_u64(const void* a, const void* b) {
  const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

static int cmp_i32(const void* a, const void* b) {
  const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Undirected simple graph as sorted adjacency lists. */
typedef struct {
  int64_t n, m;
  int64_t* off;  /* [n+1] */
  int32_t* adj;  /* [2m], each row sorted ascending */
} og_graph;

static void og_free(og_graph* g) {
  free(g->off);
  free(g->adj);
  g->off = NULL;
  g->adj = NULL;
}

/* The edge set E as sorted unique keys min << 32 | max (symmetrised, self
 * loops and duplicate pairs dropped). Returns |E|, -1 on an id outside
 * [0,n), -2 on allocation failure; *out receives the array (caller frees). */
static int64_t og_keys(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst, uint64_t** out) {
  uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m_raw > 0 ? m_raw : 1));
  if (!key) return -2;
  int64_t k = 0;
  for (int64_t e = 0; e < m_raw; ++e) {
    int64_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) { free(key); return -1; }
    if (u == v) continue;
    int64_t a = u < v ? u : v, b = u < v ? v : u;
    key[k++] = ((uint64_t)a << 32) | (uint64_t)b;
  }
  qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
  int64_t m = 0;
  for (int64_t i = 0; i < k; ++i)
    if (i == 0 || key[i] != key[i - 1]) key[m++] = key[i];
  *out = key;
  return m;
}

/* Symmetrise, drop self loops and duplicate pairs. Returns 0, -1 on an id
 * outside [0,n), -2 on allocation failure. */
static int og_build(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst, og_graph* g) {
  memset(g, 0, sizeof(*g));
  g->n = n;
  uint64_t* key = NULL;
  const int64_t m = og_keys(n, m_raw, src, dst, &key);
  if (m < 0) return (int)m;
  g->m = m;
  g->off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  g->adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * m > 0 ? 2 * m : 1));
  if (!g->off || !g->adj) { free(key); og_free(g); return -2; }
  for (int64_t i = 0; i < m; ++i) {
    g->off[(key[i] >> 32) + 1]++;
    g->off[(key[i] & 0xffffffffu) + 1]++;
  }
  for (int64_t v = 0; v < n; ++v) g->off[v + 1] += g->off[v];
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!cur) { free(key); og_free(g); return -2; }
  memcpy(cur, g->off, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; ++i) {
    int64_t a = (int64_t)(key[i] >> 32), b = (int64_t)(key[i] & 0xffffffffu);
    g->adj[cur[a]++] = (int32_t)b;
    g->adj[cur[b]++] = (int32_t)a;
  }
  free(cur);
  free(key);
  for (int64_t v = 0; v < n; ++v)
    qsort(g->adj + g->off[v], (size_t)(g->off[v + 1] - g->off[v]), sizeof(int32_t), cmp_i32);
  return 0;
}

/* rank(a) < rank(b) */
static inline int og_below(const og_graph* g, int order_mode, int64_t a, int64_t b) {
  if (order_mode == 0) return a < b;
  int64_t da = g->off[a + 1] - g->off[a], db = g->off[b + 1] - g->off[b];
  return da < db || (da == db && a < b);
}

/* Node-iterator count from the lowest-ranked vertices v = offset, offset +
 * stride, ... (stride 1, offset 0: the whole graph); T must be zeroed. */
static uint64_t og_count_from(const og_graph* g, int order_mode, int nthreads, int64_t stride, int64_t offset,
                              uint64_t* T) {
  const int64_t n = g->n;
  uint64_t total = 0;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  const int64_t nv = offset < n ? (n - offset + stride - 1) / stride : 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : total)
  {
    int64_t* mark = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < nv; ++i) {
      const int64_t v = offset + i * stride;
      for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) mark[g->adj[p]] = v + 1;
      for (int64_t p = g->off[v]; p < g->off[v + 1]; ++p) {
        const int64_t u = g->adj[p];
        if (!og_below(g, order_mode, v, u)) continue;
        for (int64_t q = g->off[u]; q < g->off[u + 1]; ++q) {
          const int64_t w = g->adj[q];
          if (!og_below(g, order_mode, u, w)) continue;
          if (mark[w] != v + 1) continue;
          /* triangle {v, u, w}, met only here */
#pragma omp atomic
          T[v] += 1;
#pragma omp atomic
          T[u] += 1;
#pragma omp atomic
          T[w] += 1;
          total += 1;
        }
      }
    }
    free(mark);
  }
  return total;
}

static uint64_t og_count(const og_graph* g, int order_mode, int nthreads, uint64_t* T) {
  return og_count_from(g, order_mode, nthreads, 1, 0, T);
}

static void og_cc(const og_graph* g, const uint64_t* T, double* cc, double* avg) {
  double sum = 0.0;
  for (int64_t v = 0; v < g->n; ++v) {
    const int64_t d = g->off[v + 1] - g->off[v];
    const double c = d >= 2 ? 2.0 * (double)T[v] / ((double)d * (double)(d - 1)) : 0.0;
    if (cc) cc[v] = c;
    sum += c;
  }
  *avg = g->n > 0 ? sum / (double)g->n : 0.0;
}

/*
 * Per-node triangle counts T[n], per-node clustering coefficients cc[n]
 * (FP64), degrees deg[n], the total triangle count, the average clustering
 * coefficient over all n ids, and the number of undirected simple edges.
 * Any output pointer except total/avg/m_out may be NULL.
 * Returns 0; -1 if an id is outside [0,n); -2 on allocation failure.
 */
int oracle_count(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst,
                 int order_mode, int nthreads, uint64_t* T, double* cc, int64_t* deg,
                 uint64_t* total, double* avg, int64_t* m_out) {
  og_graph g;
  int rc = og_build(n, m_raw, src, dst, &g);
  if (rc) return rc;
  uint64_t* t = T ? T : (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  if (!t) { og_free(&g); return -2; }
  memset(t, 0, sizeof(uint64_t) * (size_t)n);
  *total = og_count(&g, order_mode, nthreads, t);
  og_cc(&g, t, cc, avg);
  if (deg)
    for (int64_t v = 0; v < n; ++v) deg[v] = g.off[v + 1] - g.off[v];
  if (m_out) *m_out = g.m;
  if (!T) free(t);
  og_free(&g);
  return 0;
}

/*
 * Timing of the oracle on a node sample of a large graph: the graph build
 * (symmetrise, dedup, sorted rows) over all pairs, timed on its own, then the
 * node iterator from the lowest-ranked vertices v with v % stride == offset
 * only, on nthreads threads, timed on its own; then, if stride1 > 0, the
 * same from v % stride1 == offset on one thread, timed on its own. *tri and
 * *tri1 receive the triangles whose lowest-ranked vertex is in each sample
 * (summed over offset = 0 .. stride-1 that is the total).
 * Returns 0; -1 for an id outside [0,n); -2 on allocation failure; -3 for a
 * bad stride or offset.
 */
int oracle_count_timed(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst, int order_mode,
                       int nthreads, int64_t stride, int64_t offset, int64_t stride1, uint64_t* tri, uint64_t* tri1,
                       int64_t* m_out, double* build_s, double* count_s, double* count1_s) {
  if (stride < 1 || offset < 0 || offset >= stride || stride1 < 0 || (stride1 > 0 && offset >= stride1)) return -3;
  og_graph g;
  const double t0 = omp_get_wtime();
  int rc = og_build(n, m_raw, src, dst, &g);
  if (rc) return rc;
  const double t1 = omp_get_wtime();
  uint64_t* t = (uint64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
  if (!t) { og_free(&g); return -2; }
  *tri = og_count_from(&g, order_mode, nthreads, stride, offset, t);
  const double t2 = omp_get_wtime();
  *tri1 = 0;
  *count1_s = 0.0;
  if (stride1 > 0) {
    memset(t, 0, sizeof(uint64_t) * (size_t)n);
    *tri1 = og_count_from(&g, order_mode, 1, stride1, offset, t);
    *count1_s = omp_get_wtime() - t2;
  }
  *build_s = t1 - t0;
  *count_s = t2 - t1;
  if (m_out) *m_out = g.m;
  free(t);
  og_free(&g);
  return 0;
}

/*
 * Induced subgraph G[S] (subgraph extraction, Table of analytics methods;
 * node ids are kept, Section 3.1): the edges of G with both ends in S.
 * Results are indexed by position in S: T[k], cc[k]; the average is over
 * the k = |S| nodes. Returns -3 if S holds a repeated or invalid id.
 */
int oracle_induced(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst,
                   int64_t k, const int32_t* S, int nthreads, uint64_t* T, double* cc,
                   uint64_t* total, double* avg, int64_t* m_out) {
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!pos) return -2;
  for (int64_t v = 0; v < n; ++v) pos[v] = -1;
  for (int64_t i = 0; i < k; ++i) {
    if (S[i] < 0 || S[i] >= n || pos[S[i]] >= 0) { free(pos); return -3; }
    pos[S[i]] = i;
  }
  int64_t cnt = 0;
  for (int64_t e = 0; e < m_raw; ++e) {
    if (src[e] < 0 || dst[e] < 0 || src[e] >= n || dst[e] >= n) { free(pos); return -1; }
    if (pos[src[e]] >= 0 && pos[dst[e]] >= 0) ++cnt;
  }
  int32_t* s2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt > 0 ? cnt : 1));
  int32_t* d2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cnt > 0 ? cnt : 1));
  if (!s2 || !d2) { free(pos); free(s2); free(d2); return -2; }
  cnt = 0;
  for (int64_t e = 0; e < m_raw; ++e)
    if (pos[src[e]] >= 0 && pos[dst[e]] >= 0) {
      s2[cnt] = (int32_t)pos[src[e]];
      d2[cnt] = (int32_t)pos[dst[e]];
      ++cnt;
    }
  free(pos);
  int rc = oracle_count(k, cnt, s2, d2, 0, nthreads, T, cc, NULL, total, avg, m_out);
  free(s2);
  free(d2);
  return rc;
}

/*
 * T(s) and d(s) for a few sampled nodes, straight from the definition and
 * the raw edge list, without building the graph: N(s) is collected from the
 * pairs that touch s, and T(s) is the number of distinct undirected pairs
 * {a,b}, a != b, among the input edges with both a and b in N(s).
 * Samples must be distinct ids in [0,n). Single-threaded.
 */
int oracle_sampled(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst,
                   int64_t ns, const int32_t* samples, uint64_t* T, int64_t* deg) {
  int rc = 0;
  int64_t* sid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* noff = (int64_t*)calloc((size_t)ns + 1, sizeof(int64_t));
  int64_t* inv_off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* nb = NULL;
  int32_t* inv = NULL;
  int64_t* poff = NULL;
  uint64_t* pairs = NULL;
  if (!sid || !noff || !inv_off) { rc = -2; goto done; }
  for (int64_t v = 0; v < n; ++v) sid[v] = -1;
  for (int64_t i = 0; i < ns; ++i) {
    if (samples[i] < 0 || samples[i] >= n || sid[samples[i]] >= 0) { rc = -3; goto done; }
    sid[samples[i]] = i;
  }
  /* N(s): raw neighbour occurrences, then sort + unique */
  for (int64_t e = 0; e < m_raw; ++e) {
    const int32_t u = src[e], v = dst[e];
    if (u < 0 || v < 0 || u >= n || v >= n) { rc = -1; goto done; }
    if (u == v) continue;
    if (sid[u] >= 0) noff[sid[u] + 1]++;
    if (sid[v] >= 0) noff[sid[v] + 1]++;
  }
  for (int64_t i = 0; i < ns; ++i) noff[i + 1] += noff[i];
  nb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(noff[ns] > 0 ? noff[ns] : 1));
  if (!nb) { rc = -2; goto done; }
  {
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    if (!cur) { rc = -2; goto done; }
    memcpy(cur, noff, sizeof(int64_t) * (size_t)ns);
    for (int64_t e = 0; e < m_raw; ++e) {
      const int32_t u = src[e], v = dst[e];
      if (u == v) continue;
      if (sid[u] >= 0) nb[cur[sid[u]]++] = v;
      if (sid[v] >= 0) nb[cur[sid[v]]++] = u;
    }
    free(cur);
  }
  for (int64_t i = 0; i < ns; ++i) {
    int32_t* row = nb + noff[i];
    int64_t len = noff[i + 1] - noff[i], d = 0;
    qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
    for (int64_t j = 0; j < len; ++j)
      if (j == 0 || row[j] != row[j - 1]) row[d++] = row[j];
    deg[i] = d;
  }
  /* inverse lists: for node x, the samples whose neighbourhood holds x */
  for (int64_t i = 0; i < ns; ++i)
    for (int64_t j = 0; j < deg[i]; ++j) inv_off[nb[noff[i] + j] + 1]++;
  for (int64_t v = 0; v < n; ++v) inv_off[v + 1] += inv_off[v];
  inv = (int32_t*)malloc(sizeof(int32_t) * (size_t)(inv_off[n] > 0 ? inv_off[n] : 1));
  if (!inv) { rc = -2; goto done; }
  {
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!cur) { rc = -2; goto done; }
    memcpy(cur, inv_off, sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < ns; ++i)
      for (int64_t j = 0; j < deg[i]; ++j) {
        const int32_t x = nb[noff[i] + j];
        inv[cur[x]++] = (int32_t)i; /* ascending sample index */
      }
    free(cur);
  }
  /* edges {a,b} with both ends in N(s): count, fill, then sort + unique */
  poff = (int64_t*)calloc((size_t)ns + 1, sizeof(int64_t));
  if (!poff) { rc = -2; goto done; }
  for (int pass = 0; pass < 2; ++pass) {
    int64_t* cur = NULL;
    if (pass == 1) {
      for (int64_t i = 0; i < ns; ++i) poff[i + 1] += poff[i];
      pairs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(poff[ns] > 0 ? poff[ns] : 1));
      cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
      if (!pairs || !cur) { free(cur); rc = -2; goto done; }
      memcpy(cur, poff, sizeof(int64_t) * (size_t)ns);
    }
    for (int64_t e = 0; e < m_raw; ++e) {
      const int64_t a = src[e], b = dst[e];
      if (a == b) continue;
      int64_t i = inv_off[a], j = inv_off[b];
      const int64_t ie = inv_off[a + 1], je = inv_off[b + 1];
      while (i < ie && j < je) {
        if (inv[i] < inv[j]) ++i;
        else if (inv[i] > inv[j]) ++j;
        else {
          if (pass == 0) poff[inv[i] + 1]++;
          else {
            const uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
            pairs[cur[inv[i]]++] = (lo << 32) | hi;
          }
          ++i;
          ++j;
        }
      }
    }
    free(cur);
  }
  for (int64_t i = 0; i < ns; ++i) {
    uint64_t* row = pairs + poff[i];
    const int64_t len = poff[i + 1] - poff[i];
    qsort(row, (size_t)len, sizeof(uint64_t), cmp_u64);
    uint64_t t = 0;
    for (int64_t j = 0; j < len; ++j)
      if (j == 0 || row[j] != row[j - 1]) ++t;
    T[i] = t;
  }
done:
  free(sid);
  free(noff);
  free(inv_off);
  free(nb);
  free(inv);
  free(poff);
  free(pairs);
  return rc;
}

/*
 * Edge-existence tests (IsEdge, among the graph methods of Section 4; the
 * paper tests an edge by searching a node's sorted neighbour vector,
 * Section 5.1, at O(log deg_max) in its complexity table, and times random
 * tests in Section 6.2). Written as the definition: out[i] = 1 when
 * {qu[i], qv[i]} is in E, 0 when it is not (a pair (v, v) never is, E has
 * no self loops), 0xFF when qu[i] or qv[i] lies outside [0,n); E's sorted
 * keys are searched with the C library's bsearch. Returns 0, -1 if an input
 * pair holds an id outside [0,n), -2 on allocation failure.
 */
int oracle_has_edges(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst,
                     int64_t q, const int32_t* qu, const int32_t* qv, uint8_t* out) {
  uint64_t* key = NULL;
  const int64_t m = og_keys(n, m_raw, src, dst, &key);
  if (m < 0) return (int)m;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < q; ++i) {
    const int64_t u = qu[i], v = qv[i];
    if (u < 0 || v < 0 || u >= n || v >= n) {
      out[i] = 0xFF;
      continue;
    }
    if (u == v) {
      out[i] = 0;
      continue;
    }
    const uint64_t k = ((uint64_t)(u < v ? u : v) << 32) | (uint64_t)(u < v ? v : u);
    out[i] = bsearch(&k, key, (size_t)m, sizeof(uint64_t), cmp_u64) != NULL;
  }
  free(key);
  return 0;
}

/*
 * Core numbers (k-core analysis, among the analytics methods of Section 4;
 * Section 5 names the decomposition algorithm of Batagelj and Zaversnik
 * and the operations it needs: visit the nodes, read a node's degree,
 * delete it). The k-core is the largest subgraph whose nodes all have
 * degree >= k; core[v] is the largest k whose k-core holds v.
 * The bucket algorithm: nodes sorted by current degree; repeatedly take the
 * node v of smallest current degree (its core number is that degree) and
 * lower by one the current degree of every neighbour still above it,
 * moving that neighbour one bucket down. O(n + m).
 * k_stop >= 0: core[v] = min(core number, k_stop), so the k_stop-core is
 * { v : core[v] == k_stop }. Returns 0, -1 on an id outside [0,n), -2 on
 * allocation failure.
 */
int oracle_core(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst, int32_t k_stop,
                int32_t* core) {
  og_graph g;
  int rc = og_build(n, m_raw, src, dst, &g);
  if (rc) return rc;
  int64_t md = 0;
  int64_t* d = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* pos = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* vert = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t v = 0; v < n && d; ++v) {
    d[v] = g.off[v + 1] - g.off[v];
    if (d[v] > md) md = d[v];
  }
  int64_t* bin = (int64_t*)calloc((size_t)md + 2, sizeof(int64_t)); /* bin[x]: first position of degree x */
  if (!d || !pos || !vert || !bin) { rc = -2; goto done; }
  for (int64_t v = 0; v < n; ++v) bin[d[v] + 1]++;
  for (int64_t x = 0; x <= md; ++x) bin[x + 1] += bin[x];
  {
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(md + 1));
    if (!fill) { rc = -2; goto done; }
    memcpy(fill, bin, sizeof(int64_t) * (size_t)(md + 1));
    for (int64_t v = 0; v < n; ++v) {
      pos[v] = fill[d[v]]++;
      vert[pos[v]] = v;
    }
    free(fill);
  }
  for (int64_t i = 0; i < n; ++i) {
    const int64_t v = vert[i];
    for (int64_t p = g.off[v]; p < g.off[v + 1]; ++p) {
      const int64_t u = g.adj[p];
      if (d[u] > d[v]) {
        /* swap u with the first node of its bucket, then shrink the bucket */
        const int64_t du = d[u], pu = pos[u], pw = bin[du], w = vert[pw];
        if (u != w) {
          pos[u] = pw;
          vert[pw] = u;
          pos[w] = pu;
          vert[pu] = w;
        }
        bin[du]++;
        d[u]--;
      }
    }
  }
  for (int64_t v = 0; v < n; ++v) core[v] = (int32_t)(k_stop >= 0 && d[v] > k_stop ? k_stop : d[v]);
done:
  free(d);
  free(pos);
  free(vert);
  free(bin);
  og_free(&g);
  return rc;
}

/*
 * Number of 4-cliques (clique detection, among the graph-motif methods of
 * Section 4; the same counting of small complete subgraphs as the
 * triangles above, one size up). Each 4-clique {u, w, x, z} with
 * rank(u) < rank(w) < rank(x) < rank(z) is met once, at u: w is a
 * neighbour of u ranked above it, x a neighbour of w ranked above w and
 * marked as a neighbour of u, z a neighbour of x ranked above x and marked
 * as a common neighbour of u and w. order_mode as for oracle_count.
 * Returns 0, -1 on an id outside [0,n), -2 on allocation failure.
 */
int oracle_k4(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst, int order_mode, int nthreads,
              uint64_t* total) {
  og_graph g;
  int rc = og_build(n, m_raw, src, dst, &g);
  if (rc) return rc;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  uint64_t count = 0;
  int failed = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : count)
  {
    int64_t* m1 = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t)); /* neighbour of u above it */
    int64_t* m2 = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t)); /* common with w */
    if (!m1 || !m2) {
#pragma omp atomic write
      failed = 1;
    } else {
      int64_t stamp = 0;
#pragma omp for schedule(dynamic, 64)
      for (int64_t u = 0; u < n; ++u) {
        for (int64_t p = g.off[u]; p < g.off[u + 1]; ++p)
          if (og_below(&g, order_mode, u, g.adj[p])) m1[g.adj[p]] = u + 1;
        for (int64_t p = g.off[u]; p < g.off[u + 1]; ++p) {
          const int64_t w = g.adj[p];
          if (!og_below(&g, order_mode, u, w)) continue;
          ++stamp;
          for (int64_t q = g.off[w]; q < g.off[w + 1]; ++q) {
            const int64_t x = g.adj[q];
            if (og_below(&g, order_mode, w, x) && m1[x] == u + 1) m2[x] = stamp;
          }
          for (int64_t q = g.off[w]; q < g.off[w + 1]; ++q) {
            const int64_t x = g.adj[q];
            if (m2[x] != stamp) continue;
            for (int64_t r = g.off[x]; r < g.off[x + 1]; ++r) {
              const int64_t z = g.adj[r];
              if (og_below(&g, order_mode, x, z) && m2[z] == stamp) count += 1;
            }
          }
        }
      }
    }
    free(m1);
    free(m2);
  }
  og_free(&g);
  if (failed) return -2;
  *total = count;
  return 0;
}

/*
 * SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the state advances by the 64-bit golden-ratio
 * increment, and each output is the state passed through two xor-shift /
 * multiply steps and a final xor-shift.
 */
static const uint64_t sm_gamma = 0x9E3779B97F4A7C15ULL;

static uint64_t sm_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* The first `count` outputs of SplitMix64 started from state `state`. */
int oracle_splitmix64(uint64_t state, int64_t count, uint64_t* out) {
  for (int64_t i = 0; i < count; ++i) {
    state += sm_gamma;
    out[i] = sm_out(state);
  }
  return 0;
}

/*
 * R-MAT edges (the paper's table of graph generators, Section 4, cites
 * Chakrabarti, Zhan and Faloutsos, SDM 2004), with per-level noise on the
 * quadrant probabilities, as defined for the GPU generator:
 *
 *   word(c)  = c-th output (c = 1, 2, ...) of SplitMix64 started from state
 *              S = out(seed + gamma * 12), i.e. out(S + gamma * c)   (stream 11)
 *   edge e   = `scale` quadrant choices, most significant bit first; at level
 *              l, with k = 2 (e * scale + l):
 *     h_q    = bits 16q .. 16q+15 of word(k + 1), q = 0..3
 *     p_q    = base_q * (1 + noise * (2 h_q / 65535 - 1))          (FP64)
 *     x      = (word(k + 2) >> 11) * 2^-53 * (p_0 + p_1 + p_2 + p_3)
 *     q      = first q in 0..2 with x < p_0 + ... + p_q, else 3
 *     src bit = q >> 1, dst bit = q & 1   (a = (0,0), b = (0,1), c = (1,0), d = (1,1))
 *   perm     = optional relabelling: both ends id -> perm[id].
 *
 * Self loops and duplicate pairs are kept. The edges are the k indices in
 * idx (all of 0..k-1 when idx is NULL). Every FP64 operation is a separately
 * rounded IEEE operation in the order written above (sums left to right).
 * Returns 0, -1 on a bad scale.
 */
int oracle_rmat(int scale, double a, double b, double c, double d, double noise, uint64_t seed, int64_t k,
                const int64_t* idx, const int32_t* perm, int32_t* src, int32_t* dst) {
  if (scale < 1 || scale > 30) return -1;
  const double base[4] = {a, b, c, d};
  const uint64_t S = sm_out(seed + sm_gamma * 12u);
  for (int64_t i = 0; i < k; ++i) {
    const uint64_t e = idx ? (uint64_t)idx[i] : (uint64_t)i;
    uint32_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      const uint64_t kk = 2u * (e * (uint64_t)scale + (uint64_t)l);
      const uint64_t w1 = sm_out(S + sm_gamma * (kk + 1u));
      const uint64_t w2 = sm_out(S + sm_gamma * (kk + 2u));
      double p[4];
      for (int q = 0; q < 4; ++q) {
        const double h = (double)((w1 >> (16 * q)) & 0xFFFFu);
        p[q] = base[q] * (1.0 + noise * (2.0 * h / 65535.0 - 1.0));
      }
      const double x = (double)(w2 >> 11) * 0x1.0p-53 * (((p[0] + p[1]) + p[2]) + p[3]);
      int q;
      if (x < p[0]) q = 0;
      else if (x < p[0] + p[1]) q = 1;
      else if (x < (p[0] + p[1]) + p[2]) q = 2;
      else q = 3;
      u = (u << 1) | (uint32_t)(q >> 1);
      v = (v << 1) | (uint32_t)(q & 1);
    }
    src[i] = perm ? perm[u] : (int32_t)u;
    dst[i] = perm ? perm[v] : (int32_t)v;
  }
  return 0;
}

/*
 * Number of 5-cliques (clique detection, the paper's Section 4 table of
 * graph-motif methods): every 5-clique has one vertex u of lowest rank, and
 * its other four vertices w < x < y < z (by rank) satisfy w in N+(u),
 * x in C1 = N+(u) ∩ N+(w), y in C2 = C1 ∩ N+(x), z in C2 ∩ N+(y), where N+(v)
 * is the set of neighbours ranked above v. The count is the sum over u, w,
 * x, y of |N+(y) ∩ C2|: three marker levels (N+(u), C1, C2) over a plain
 * node iterator, with either rank order (order_mode as for oracle_k4).
 * Returns 0, -1 on an id outside [0,n), -2 on allocation failure.
 */
int oracle_k5(int64_t n, int64_t m_raw, const int32_t* src, const int32_t* dst, int order_mode, int nthreads,
              uint64_t* total) {
  og_graph g;
  int rc = og_build(n, m_raw, src, dst, &g);
  if (rc) return rc;
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  uint64_t count = 0;
  int failed = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : count)
  {
    int64_t* m1 = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t)); /* in N+(u) */
    int64_t* m2 = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t)); /* in C1 */
    int64_t* m3 = (int64_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t)); /* in C2 */
    if (!m1 || !m2 || !m3) {
#pragma omp atomic write
      failed = 1;
    } else {
      int64_t s2 = 0, s3 = 0;
#pragma omp for schedule(dynamic, 64)
      for (int64_t u = 0; u < n; ++u) {
        for (int64_t p = g.off[u]; p < g.off[u + 1]; ++p)
          if (og_below(&g, order_mode, u, g.adj[p])) m1[g.adj[p]] = u + 1;
        for (int64_t p = g.off[u]; p < g.off[u + 1]; ++p) {
          const int64_t w = g.adj[p];
          if (!og_below(&g, order_mode, u, w)) continue;
          ++s2;
          for (int64_t q = g.off[w]; q < g.off[w + 1]; ++q) {
            const int64_t x = g.adj[q];
            if (og_below(&g, order_mode, w, x) && m1[x] == u + 1) m2[x] = s2;
          }
          for (int64_t q = g.off[w]; q < g.off[w + 1]; ++q) {
            const int64_t x = g.adj[q];
            if (m2[x] != s2) continue;
            ++s3;
            for (int64_t r = g.off[x]; r < g.off[x + 1]; ++r) {
              const int64_t y = g.adj[r];
              if (og_below(&g, order_mode, x, y) && m2[y] == s2) m3[y] = s3;
            }
            for (int64_t r = g.off[x]; r < g.off[x + 1]; ++r) {
              const int64_t y = g.adj[r];
              if (m3[y] != s3) continue;
              for (int64_t t = g.off[y]; t < g.off[y + 1]; ++t) {
                const int64_t z = g.adj[t];
                if (og_below(&g, order_mode, y, z) && m3[z] == s3) count += 1;
              }
            }
          }
        }
      }
    }
    free(m1);
    free(m2);
    free(m3);
  }
  og_free(&g);
  if (failed) return -2;
  *total = count;
  return 0;
}

/* floor(w * N / 2^64): the high word of the 128-bit product. */
static uint64_t mul_hi(uint64_t w, uint64_t N) { return (uint64_t)(((unsigned __int128)w * N) >> 64); }

/* Largest i in [0, n-2] with i n - i(i+1)/2 <= t (binary search). */
static int64_t pair_row(int64_t n, uint64_t t) {
  int64_t lo = 0, hi = n - 2;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if ((uint64_t)(mid * n - mid * (mid + 1) / 2) <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

/*
 * Erdos-Renyi G(n, m) (the paper's table of graph generators, Section 4,
 * names the G(n, m) model), as defined for the GPU generator: a uniform
 * random m-subset of the N = n(n-1)/2 node pairs, by rejecting repeats in a
 * counter-based sequence of uniform pair indices:
 *
 *   word(c) = out(S + gamma c), c = 1, 2, ...; S = out(seed + gamma * 13)
 *   x_k     = floor(word(k + 1) N / 2^64), k = 0, 1, ...
 *   edges   = the first m distinct values of x_0, x_1, ..., in draw order;
 *             pair index t is the pair (i, j), i < j, with
 *             t = i n - i(i+1)/2 + (j - i - 1) (row by row), written as
 *             (i, j), or (j, i) when the low bit of its draw's word is 1.
 *
 * Returns 0; -1 for n outside [0, 2^31) or m outside [0, N]; -2 on
 * allocation failure; -3 if the draws run past a guard far above what m
 * distinct values need.
 */
int oracle_er(int64_t n, int64_t m, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n < 0 || n > 0x7fffffffLL) return -1;
  const uint64_t N = n > 1 ? (uint64_t)n * (uint64_t)(n - 1) / 2 : 0;
  if (m < 0 || (uint64_t)m > N) return -1;
  if (m == 0) return 0;
  uint64_t cap = 1;
  while (cap < 2 * (uint64_t)m) cap <<= 1;
  uint64_t* set = (uint64_t*)malloc(sizeof(uint64_t) * cap); /* value + 1; 0 = empty */
  if (!set) return -2;
  memset(set, 0, sizeof(uint64_t) * cap);
  const uint64_t S = sm_out(seed + sm_gamma * 13u);
  int64_t got = 0;
  /* a guard only: the draws a valid run needs stay far below this */
  const uint64_t draw_cap = 64u * (N + (uint64_t)m) + (1u << 20);
  for (uint64_t k = 0; got < m; ++k) {
    if (k >= draw_cap) { free(set); return -3; }
    const uint64_t w = sm_out(S + sm_gamma * (k + 1u));
    const uint64_t x = mul_hi(w, N);
    uint64_t h = (x * 0x9E3779B97F4A7C15ULL) & (cap - 1);
    int seen = 0;
    while (set[h]) {
      if (set[h] == x + 1) { seen = 1; break; }
      h = (h + 1) & (cap - 1);
    }
    if (seen) continue;
    set[h] = x + 1;
    const int64_t i = pair_row(n, x);
    const int64_t j = (int64_t)(x - (uint64_t)(i * n - i * (i + 1) / 2)) + i + 1;
    src[got] = (int32_t)((w & 1u) ? j : i);
    dst[got] = (int32_t)((w & 1u) ? i : j);
    ++got;
  }
  free(set);
  return 0;
}

/*
 * Barabasi-Albert (the paper's table of graph generators, Section 4, names
 * preferential attachment), as defined for the GPU generator, with k
 * distinct targets per node:
 *
 *   nodes 0..k form the clique K_{k+1}: edges e = 0 .. k(k+1)/2 - 1 are its
 *   pairs (i, j), i < j, in lexicographic order (source i, target j);
 *   node v > k adds edges e = E_v + j, j = 0 .. k-1, with source v, where
 *   E_v = k(k+1)/2 + (v - k - 1) k is the number of edges before v's.
 *   Edge e' holds its source at endpoint position 2e' and its target at
 *   2e' + 1; the target of edge e = E_v + j is the node at position
 *     r = floor(word((e << 20) + a + 1) 2 E_v / 2^64)
 *   (S = out(seed + gamma * 14)) for the first attempt a = 0, 1, ... whose
 *   node differs from the targets of v's edges j' < j. Each position holds
 *   one endpoint, so a node is drawn with probability proportional to its
 *   degree among the edges before v's.
 *
 * src, dst: m = k(k+1)/2 + (n - k - 1) k entries. Returns 0; -1 unless
 * 1 <= k <= 255 and k < n < 2^31; -3 if an edge needs 2^20 attempts.
 */
int oracle_ba(int64_t n, int32_t k, uint64_t seed, int32_t* src, int32_t* dst) {
  if (k < 1 || k > 255 || n < k + 1 || n > 0x7fffffffLL) return -1;
  const int64_t es = (int64_t)k * (k + 1) / 2;
  int64_t e = 0;
  for (int32_t i = 0; i <= k; ++i)
    for (int32_t j = i + 1; j <= k; ++j) {
      src[e] = i;
      dst[e] = j;
      ++e;
    }
  const uint64_t S = sm_out(seed + sm_gamma * 14u);
  for (int64_t v = k + 1; v < n; ++v) {
    const int64_t ev = es + (v - k - 1) * (int64_t)k;
    for (int32_t j = 0; j < k; ++j) {
      const int64_t ej = ev + j;
      int32_t c = -1;
      for (uint64_t a = 0;; ++a) {
        if (a >= (1u << 20)) return -3;
        const uint64_t r = mul_hi(sm_out(S + sm_gamma * (((uint64_t)ej << 20) + a + 1u)), 2u * (uint64_t)ev);
        c = (r & 1u) ? dst[r >> 1] : src[r >> 1];
        int dup = 0;
        for (int32_t q = 0; q < j; ++q) dup |= dst[ev + q] == c;
        if (!dup) break;
      }
      src[ej] = (int32_t)v;
      dst[ej] = c;
    }
  }
  return 0;
}

/* Wall-clock seconds (monotonic), for timing the oracle in the benchmark. */
double oracle_wtime(void) { return omp_get_wtime(); }

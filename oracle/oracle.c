/*
 * oracle.c -- plain, slow CPU reference for single-source shortest paths with
 * triangle-based edge pruning.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the HIP library is
 * compared against; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or helper with
 * the GPU library and must never be linked into it.
 *
 * Problem (Sec. I, LP formulation): a directed graph G(V,E) with a source S
 * and a nonnegative cost w on every arc; d(v) is the minimum over S->v paths
 * of the summed cost (the optimum of the path LP; its dual is the potential
 * d with d(v) <= d(u) + w(u,v) on every arc).  Unreachable vertices have
 * d(v) = infinity.
 *
 * Conventions fixed here (the paper is silent on them):
 *   - graphs are CSR: row_ptr[n+1], col[m]; edge id e is the position in col;
 *   - integer weights are uint32, path sums are accumulated in uint64;
 *   - fp32 weights accumulate left to right from the source in float
 *     (round-to-nearest-even, no contraction): d(v) = fl32(d(u) + w);
 *   - pred_edge(v) for reached v != S is the smallest edge id e = (u,v) that
 *     is tight, d(u) + w_e == d(v) with d(u) finite; pred_edge(S) = -1 and
 *     unreachable vertices have -1;
 *   - Trishla (Sec. III-B, Alg. 1) marks edge e = (u,x,W) for deletion when a
 *     middle vertex y, y != u and y != x, has arcs (u,y,w1) and (y,x,w2) with
 *     w1 + w2 < W (strict).  The test is evaluated on the input graph for all
 *     edges at once (no edge's deletion influences another edge's test).
 *     Scope GLOBAL lets y be any vertex; scope LOCAL demands that y lies in
 *     the partition of u (1D block partition of Sec. III-A with block size
 *     ceil(n/P)).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define U64_INF UINT64_MAX

/* ------------------------------------------------------------------------ */
/* Binary min-heap of (uint64 key, vertex) with lazy deletion.              */
/* Nonnegative IEEE floats order like their bit patterns, so fp32 / fp64     */
/* distances are keyed by their bits.                                        */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t key; int32_t v; } hitem;
typedef struct { hitem *a; int64_t size; } heap_t;

static void heap_push(heap_t *h, uint64_t key, int32_t v) {
  int64_t i = h->size++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->a[p].key <= key) break;
    h->a[i] = h->a[p];
    i = p;
  }
  h->a[i].key = key;
  h->a[i].v = v;
}

static hitem heap_pop(heap_t *h) {
  hitem top = h->a[0];
  hitem last = h->a[--h->size];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= h->size) break;
    if (c + 1 < h->size && h->a[c + 1].key < h->a[c].key) c++;
    if (last.key <= h->a[c].key) break;
    h->a[i] = h->a[c];
    i = c;
  }
  if (h->size > 0) h->a[i] = last;
  return top;
}

static uint64_t f32_key(float x) { uint32_t b; memcpy(&b, &x, 4); return b; }
static uint64_t f64_key(double x) { uint64_t b; memcpy(&b, &x, 8); return b; }

/* ------------------------------------------------------------------------ */
/* Dijkstra (binary heap).  The paper's local rule (Sec. III-C, Alg. 3):     */
/* pop the vertex of least tentative distance, relax its out-arcs.          */
/* Return 0, or -1 when out of memory.                                       */
/* ------------------------------------------------------------------------ */
int oracle_sssp_u32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const uint32_t *w, int32_t source, uint64_t *dist) {
  int64_t m = row_ptr[n];
  heap_t h;
  h.a = (hitem *)malloc(sizeof(hitem) * (size_t)(m + 1));
  char *done = (char *)calloc((size_t)n, 1);
  if (!h.a || !done) { free(h.a); free(done); return -1; }
  h.size = 0;
  for (int32_t v = 0; v < n; v++) dist[v] = U64_INF;
  dist[source] = 0;
  heap_push(&h, 0, source);
  while (h.size > 0) {
    hitem it = heap_pop(&h);
    int32_t u = it.v;
    if (done[u]) continue;
    done[u] = 1;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      uint64_t nd = dist[u] + (uint64_t)w[e];
      if (nd < dist[v]) {
        dist[v] = nd;
        heap_push(&h, nd, v);
      }
    }
  }
  free(h.a);
  free(done);
  return 0;
}

int oracle_sssp_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const float *w, int32_t source, float *dist) {
  int64_t m = row_ptr[n];
  heap_t h;
  h.a = (hitem *)malloc(sizeof(hitem) * (size_t)(m + 1));
  char *done = (char *)calloc((size_t)n, 1);
  if (!h.a || !done) { free(h.a); free(done); return -1; }
  h.size = 0;
  for (int32_t v = 0; v < n; v++) dist[v] = INFINITY;
  dist[source] = 0.0f;
  heap_push(&h, f32_key(0.0f), source);
  while (h.size > 0) {
    hitem it = heap_pop(&h);
    int32_t u = it.v;
    if (done[u]) continue;
    done[u] = 1;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      float nd = dist[u] + w[e];
      if (nd < dist[v]) {
        dist[v] = nd;
        heap_push(&h, f32_key(nd), v);
      }
    }
  }
  free(h.a);
  free(done);
  return 0;
}

int oracle_sssp_f64(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const double *w, int32_t source, double *dist) {
  int64_t m = row_ptr[n];
  heap_t h;
  h.a = (hitem *)malloc(sizeof(hitem) * (size_t)(m + 1));
  char *done = (char *)calloc((size_t)n, 1);
  if (!h.a || !done) { free(h.a); free(done); return -1; }
  h.size = 0;
  for (int32_t v = 0; v < n; v++) dist[v] = INFINITY;
  dist[source] = 0.0;
  heap_push(&h, f64_key(0.0), source);
  while (h.size > 0) {
    hitem it = heap_pop(&h);
    int32_t u = it.v;
    if (done[u]) continue;
    done[u] = 1;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      double nd = dist[u] + w[e];
      if (nd < dist[v]) {
        dist[v] = nd;
        heap_push(&h, f64_key(nd), v);
      }
    }
  }
  free(h.a);
  free(done);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Bellman-Ford, brute force: n-1 full sweeps over every arc (plus one more  */
/* that must change nothing).  Used only to pin Dijkstra on tiny graphs.     */
/* ------------------------------------------------------------------------ */
int oracle_bellman_ford_u32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                            const uint32_t *w, int32_t source, uint64_t *dist) {
  for (int32_t v = 0; v < n; v++) dist[v] = U64_INF;
  dist[source] = 0;
  for (int32_t it = 0; it < n; it++) {
    int changed = 0;
    for (int32_t u = 0; u < n; u++) {
      if (dist[u] == U64_INF) continue;
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
        uint64_t nd = dist[u] + (uint64_t)w[e];
        if (nd < dist[col[e]]) { dist[col[e]] = nd; changed = 1; }
      }
    }
    if (!changed) return 0;
  }
  return -2; /* cannot happen with nonnegative weights */
}

int oracle_bellman_ford_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                            const float *w, int32_t source, float *dist) {
  for (int32_t v = 0; v < n; v++) dist[v] = INFINITY;
  dist[source] = 0.0f;
  for (int32_t it = 0; it <= n; it++) {
    int changed = 0;
    for (int32_t u = 0; u < n; u++) {
      if (isinf(dist[u])) continue;
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
        float nd = dist[u] + w[e];
        if (nd < dist[col[e]]) { dist[col[e]] = nd; changed = 1; }
      }
    }
    if (!changed) return 0;
  }
  return -2;
}

/* ------------------------------------------------------------------------ */
/* Predecessor post-pass: smallest tight edge id into every reached v != S.  */
/* Scanning edges in increasing id keeps the first tight one.                */
/* ------------------------------------------------------------------------ */
void oracle_pred_u32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                     const uint32_t *w, int32_t source, const uint64_t *dist,
                     int32_t *pred_edge, int32_t *pred) {
  for (int32_t v = 0; v < n; v++) { pred_edge[v] = -1; pred[v] = -1; }
  for (int32_t u = 0; u < n; u++) {
    if (dist[u] == U64_INF) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      if (v == source || pred_edge[v] != -1) continue;
      if (dist[u] + (uint64_t)w[e] == dist[v]) { pred_edge[v] = (int32_t)e; pred[v] = u; }
    }
  }
}

void oracle_pred_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                     const float *w, int32_t source, const float *dist,
                     int32_t *pred_edge, int32_t *pred) {
  for (int32_t v = 0; v < n; v++) { pred_edge[v] = -1; pred[v] = -1; }
  for (int32_t u = 0; u < n; u++) {
    if (isinf(dist[u])) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      if (v == source || pred_edge[v] != -1) continue;
      float nd = dist[u] + w[e];
      if (nd == dist[v]) { pred_edge[v] = (int32_t)e; pred[v] = u; }
    }
  }
}

void oracle_pred_f64(int32_t n, const int32_t *row_ptr, const int32_t *col,
                     const double *w, int32_t source, const double *dist,
                     int32_t *pred_edge, int32_t *pred) {
  for (int32_t v = 0; v < n; v++) { pred_edge[v] = -1; pred[v] = -1; }
  for (int32_t u = 0; u < n; u++) {
    if (isinf(dist[u])) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      if (v == source || pred_edge[v] != -1) continue;
      double nd = dist[u] + w[e];
      if (nd == dist[v]) { pred_edge[v] = (int32_t)e; pred[v] = u; }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Trishla (Sec. III-B, Alg. 1).                                             */
/* ------------------------------------------------------------------------ */

/* Exact test a + b < W for nonnegative floats: the double sum s and its     */
/* rounding error r (Knuth's two-sum) give a + b = s + r exactly.            */
static int f32_sum_lt(float a, float b, float W) {
  double x = a, y = b, s = x + y;
  double bb = s - x;
  double r = (x - (s - bb)) + (y - bb);
  if (s < (double)W) return 1;
  if (s > (double)W) return 0;
  return r < 0.0;
}

static int32_t block_of(int32_t v, int32_t bsize) { return v / bsize; }

static int32_t block_size(int32_t n, int32_t nparts) {
  if (nparts < 1) nparts = 1;
  if (nparts > n) nparts = n;
  return (n + nparts - 1) / nparts;
}

/* Triple loop over (edge, first arc, second arc).  keep[e] = 1 / 0.         */
void oracle_trishla_brute_u32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                              const uint32_t *w, int32_t local_scope, int32_t nparts,
                              uint8_t *keep) {
  int32_t bs = block_size(n, nparts);
  for (int32_t u = 0; u < n; u++) {
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t x = col[e];
      int pruned = 0;
      for (int64_t e1 = row_ptr[u]; e1 < row_ptr[u + 1] && !pruned; e1++) {
        int32_t y = col[e1];
        if (y == u || y == x) continue;
        if (local_scope && block_of(y, bs) != block_of(u, bs)) continue;
        for (int64_t e2 = row_ptr[y]; e2 < row_ptr[y + 1]; e2++) {
          if (col[e2] == x && (uint64_t)w[e1] + (uint64_t)w[e2] < (uint64_t)w[e]) {
            pruned = 1;
            break;
          }
        }
      }
      keep[e] = (uint8_t)!pruned;
    }
  }
}

void oracle_trishla_brute_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                              const float *w, int32_t local_scope, int32_t nparts,
                              uint8_t *keep) {
  int32_t bs = block_size(n, nparts);
  for (int32_t u = 0; u < n; u++) {
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t x = col[e];
      int pruned = 0;
      for (int64_t e1 = row_ptr[u]; e1 < row_ptr[u + 1] && !pruned; e1++) {
        int32_t y = col[e1];
        if (y == u || y == x) continue;
        if (local_scope && block_of(y, bs) != block_of(u, bs)) continue;
        for (int64_t e2 = row_ptr[y]; e2 < row_ptr[y + 1]; e2++) {
          if (col[e2] == x && f32_sum_lt(w[e1], w[e2], w[e])) { pruned = 1; break; }
        }
      }
      keep[e] = (uint8_t)!pruned;
    }
  }
}

/* Same definition, organised for large graphs: for every u, scatter the     */
/* cheapest two-arc cost best[x] = min_y (w(u,y) + w(y,x)) into a dense      */
/* array, then compare every arc (u,x,W) against it.  Parallel over u.       */
void oracle_trishla_mark_u32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                             const uint32_t *w, int32_t local_scope, int32_t nparts,
                             uint8_t *keep) {
  int32_t bs = block_size(n, nparts);
#pragma omp parallel
  {
    uint64_t *best = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    for (int32_t i = 0; i < n; i++) best[i] = U64_INF;
#pragma omp for schedule(dynamic, 64)
    for (int32_t u = 0; u < n; u++) {
      for (int64_t e1 = row_ptr[u]; e1 < row_ptr[u + 1]; e1++) {
        int32_t y = col[e1];
        if (y == u) continue;
        if (local_scope && block_of(y, bs) != block_of(u, bs)) continue;
        for (int64_t e2 = row_ptr[y]; e2 < row_ptr[y + 1]; e2++) {
          int32_t x = col[e2];
          if (x == y) continue;
          uint64_t c = (uint64_t)w[e1] + (uint64_t)w[e2];
          if (c < best[x]) best[x] = c;
        }
      }
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++)
        keep[e] = (uint8_t)!(best[col[e]] < (uint64_t)w[e]);
      /* reset what this row touched */
      for (int64_t e1 = row_ptr[u]; e1 < row_ptr[u + 1]; e1++) {
        int32_t y = col[e1];
        for (int64_t e2 = row_ptr[y]; e2 < row_ptr[y + 1]; e2++) best[col[e2]] = U64_INF;
      }
    }
    free(best);
  }
}

/* fp32 variant: the witness cost is kept as the exact pair (w1, w2) of the  */
/* current minimum, compared exactly.                                        */
static int f32_pair_lt(float a1, float b1, float a2, float b2) {
  /* a1 + b1 < a2 + b2, exactly: each side is its double sum s plus the     */
  /* exact rounding error r; rounding is monotone, so distinct s decide, and */
  /* equal s are decided by r.                                               */
  double s1 = (double)a1 + (double)b1, bb1 = s1 - a1;
  double r1 = ((double)a1 - (s1 - bb1)) + ((double)b1 - bb1);
  double s2 = (double)a2 + (double)b2, bb2 = s2 - a2;
  double r2 = ((double)a2 - (s2 - bb2)) + ((double)b2 - bb2);
  if (s1 != s2) return s1 < s2;
  return r1 < r2;
}

void oracle_trishla_mark_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                             const float *w, int32_t local_scope, int32_t nparts,
                             uint8_t *keep) {
  int32_t bs = block_size(n, nparts);
#pragma omp parallel
  {
    float *b1 = (float *)malloc(sizeof(float) * (size_t)n);
    float *b2 = (float *)malloc(sizeof(float) * (size_t)n);
    char *has = (char *)calloc((size_t)n, 1);
#pragma omp for schedule(dynamic, 64)
    for (int32_t u = 0; u < n; u++) {
      for (int64_t e1 = row_ptr[u]; e1 < row_ptr[u + 1]; e1++) {
        int32_t y = col[e1];
        if (y == u) continue;
        if (local_scope && block_of(y, bs) != block_of(u, bs)) continue;
        for (int64_t e2 = row_ptr[y]; e2 < row_ptr[y + 1]; e2++) {
          int32_t x = col[e2];
          if (x == y) continue;
          if (!has[x] || f32_pair_lt(w[e1], w[e2], b1[x], b2[x])) {
            has[x] = 1; b1[x] = w[e1]; b2[x] = w[e2];
          }
        }
      }
      for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
        int32_t x = col[e];
        keep[e] = (uint8_t)!(has[x] && f32_sum_lt(b1[x], b2[x], w[e]));
      }
      for (int64_t e1 = row_ptr[u]; e1 < row_ptr[u + 1]; e1++) {
        int32_t y = col[e1];
        for (int64_t e2 = row_ptr[y]; e2 < row_ptr[y + 1]; e2++) has[col[e2]] = 0;
      }
    }
    free(b1); free(b2); free(has);
  }
}

/* ------------------------------------------------------------------------ */
/* Certificate (dual of the path LP, Sec. I) for an output (dist, pred_edge).*/
/* Returns 0 when every condition holds, else a positive code and writes the */
/* offending vertex or edge to *where:                                       */
/*   1 d(S) != 0 or pred_edge(S) != -1                                        */
/*   2 infeasible arc: d(u) finite and d(v) > d(u) + w                         */
/*   3 unreached vertex with a predecessor                                    */
/*   4 reached v != S whose pred_edge is not an arc into v                    */
/*   5 pred arc not tight                                                     */
/*   6 a tight arc into v with a smaller id than pred_edge(v)                  */
/*   7 predecessor chain does not reach S (cycle)                             */
/*   8 out of memory                                                          */
/* dist uses 0xFFFFFFFF (u32) or +inf (f32) for unreachable.                  */
/* ------------------------------------------------------------------------ */
static int32_t tail_of(int32_t n, const int32_t *row_ptr, int64_t e) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {                      /* largest u with row_ptr[u] <= e */
    int32_t mid = lo + (hi - lo + 1) / 2;
    if ((int64_t)row_ptr[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static int chains_reach_source(int32_t n, const int32_t *row_ptr, int32_t source,
                               const int32_t *pred_edge, int reached_fn(int32_t, const void *),
                               const void *ctx, int64_t *where) {
  char *state = (char *)calloc((size_t)n, 1); /* 0 new, 1 on stack, 2 ok */
  int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!state || !stack) { free(state); free(stack); return 8; }
  state[source] = 2;
  for (int32_t v = 0; v < n; v++) {
    if (state[v] || !reached_fn(v, ctx)) continue;
    int32_t top = 0, x = v;
    while (state[x] == 0) {
      state[x] = 1;
      stack[top++] = x;
      x = tail_of(n, row_ptr, pred_edge[x]);
    }
    if (state[x] == 1) { *where = x; free(state); free(stack); return 7; }
    while (top > 0) state[stack[--top]] = 2;
  }
  free(state);
  free(stack);
  return 0;
}

static int reached_u32(int32_t v, const void *ctx) { return ((const uint32_t *)ctx)[v] != 0xFFFFFFFFu; }
static int reached_f32(int32_t v, const void *ctx) { return !isinf(((const float *)ctx)[v]); }

int oracle_certify_u32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const uint32_t *w, int32_t source, const uint32_t *dist,
                       const int32_t *pred_edge, int64_t *where) {
  const uint32_t INF = 0xFFFFFFFFu;
  int64_t m = row_ptr[n];
  *where = -1;
  if (dist[source] != 0 || pred_edge[source] != -1) { *where = source; return 1; }
  for (int32_t u = 0; u < n; u++) {
    if (dist[u] == INF) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      uint64_t via = (uint64_t)dist[u] + w[e];
      uint64_t dv = dist[v] == INF ? UINT64_MAX : dist[v];
      if (dv > via) { *where = e; return 2; }
      if (v != source && dv == via && e < pred_edge[v]) { *where = e; return 6; }
    }
  }
  for (int32_t v = 0; v < n; v++) {
    if (v == source) continue;
    int32_t pe = pred_edge[v];
    if (dist[v] == INF) { if (pe != -1) { *where = v; return 3; } continue; }
    if (pe < 0 || pe >= m || col[pe] != v) { *where = v; return 4; }
    int32_t u = tail_of(n, row_ptr, pe);
    if (dist[u] == INF || (uint64_t)dist[u] + w[pe] != dist[v]) { *where = v; return 5; }
  }
  return chains_reach_source(n, row_ptr, source, pred_edge, reached_u32, dist, where);
}

int oracle_certify_f32(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const float *w, int32_t source, const float *dist,
                       const int32_t *pred_edge, int64_t *where) {
  int64_t m = row_ptr[n];
  *where = -1;
  if (dist[source] != 0.0f || pred_edge[source] != -1) { *where = source; return 1; }
  for (int32_t u = 0; u < n; u++) {
    if (isinf(dist[u])) continue;
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
      int32_t v = col[e];
      float via = dist[u] + w[e];
      if (dist[v] > via) { *where = e; return 2; }
      if (v != source && dist[v] == via && e < pred_edge[v]) { *where = e; return 6; }
    }
  }
  for (int32_t v = 0; v < n; v++) {
    if (v == source) continue;
    int32_t pe = pred_edge[v];
    if (isinf(dist[v])) { if (pe != -1) { *where = v; return 3; } continue; }
    if (pe < 0 || pe >= m || col[pe] != v) { *where = v; return 4; }
    int32_t u = tail_of(n, row_ptr, pe);
    if (isinf(dist[u]) || dist[u] + w[pe] != dist[v]) { *where = v; return 5; }
  }
  return chains_reach_source(n, row_ptr, source, pred_edge, reached_f32, dist, where);
}

/* ------------------------------------------------------------------------ */
/* Gradient of L = sum_v g[v] * d(v) with respect to the arc weights, for    */
/* the shortest-path tree given by pred_edge: d(t) is the sum of the weights */
/* on the tree path S -> t, so dL/dw_e = sum of g[t] over targets t whose    */
/* tree path uses e.  Written out literally: walk every target's path.       */
/* Accumulates in double; returns 0, or 7 if a chain does not reach S.       */
/* ------------------------------------------------------------------------ */
int oracle_grad_f32(int32_t n, const int32_t *row_ptr, int32_t source,
                    const int32_t *pred_edge, const float *g, float *grad_w) {
  int64_t m = row_ptr[n];
  double *acc = (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
  if (!acc) return 8;
  int rc = 0;
  for (int32_t t = 0; t < n && !rc; t++) {
    if (g[t] == 0.0f || t == source || pred_edge[t] < 0) continue;
    int32_t x = t;
    for (int32_t steps = 0; x != source; steps++) {
      if (steps > n) { rc = 7; break; }
      int32_t e = pred_edge[x];
      if (e < 0) { rc = 7; break; }
      acc[e] += (double)g[t];
      x = tail_of(n, row_ptr, e);
    }
  }
  for (int64_t e = 0; e < m; e++) grad_w[e] = (float)acc[e];
  free(acc);
  return rc;
}

/* Number of OpenMP threads the parallel oracle routines use. */
int oracle_max_threads(void) {
  int t = 1;
#pragma omp parallel
  {
#pragma omp single
    t = omp_get_num_threads();
  }
  return t;
}

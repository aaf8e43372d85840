/*
 * oracle.c -- CPU oracle for graph best-first search with a dependency-relaxed
 * fetch schedule (FlashANNS, arXiv 2507.10070).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU search is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header or
 * helper with the GPU library and includes nothing from it.
 *
 * What it computes (paper section 4.1.1, "Data-Dependency in Traditional
 * Best-First Search", and section 4.1.2, "Dependency Relaxed Strategy"):
 *
 *   - One search step pops the closest unexpanded candidate v, reads v's
 *     record (its neighbour list), computes the distances of the neighbours to
 *     the query and inserts them into the candidate structure (section 4.1.1).
 *     The candidate structure is kept here as a sorted list of at most L
 *     entries with an "expanded" flag per entry; L is the candidate-list size
 *     that controls recall (section 5.1, evaluation metrics).
 *   - In the relaxed schedule the node fetched at step i is chosen from the
 *     candidate list as updated by step i-2 (section 4.1.2); with a staleness
 *     of `delay` the selection runs `delay` steps ahead of the processing.
 *     delay = 0 is the strict best-first search.  The staleness is read as
 *     exact (a FIFO of `delay` in-flight nodes), so results never depend on
 *     timing.
 *   - Beam width W (one node per step in the paper, W = 1 by default): each
 *     iteration selects up to W unexpanded candidates into the FIFO and
 *     processes the oldest while more than delay * W are in flight, or the
 *     oldest min(W, in flight) when nothing was selected.
 *   - Keys are (distance, id) compared lexicographically, so every key is
 *     unique and ties go to the smaller id.
 *   - The visited set is exact.
 *   - Squared L2 distance: integer vectors in 64-bit integers (exact), fp32
 *     vectors in fp64 from the fp32 inputs.
 *
 * Compressed navigation (paper section 2.2, the in-memory quantised vectors of
 * graph-indexing systems; section 8 of the oracle below): neighbours are
 * scored by a product-quantisation (PQ) distance, the candidate list is
 * ordered by it, and each expanded node's exact distance, from the
 * full-precision vector of its record, goes to a result set whose first k
 * (by exact distance, then id) are the answer.
 *
 * Parity status: pinned (see tests/test_oracle_*.py): hand-derived traces of
 * a worked example, exhaustive search on tiny inputs (L >= N gives the exact
 * top-k), a textbook heap formulation of the strict search, library
 * distances, tie-breaking fixtures and the invariants of section 4.1.3.
 *
 * Build: gcc -O2 -shared -fPIC -pthread oracle.c -o liboracle.so
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_U8 1
#define ORC_I8 2
#define ORC_F32 3

#define ORC_EINVAL (-22)
#define ORC_ENOMEM (-12)

/* ---------------------------------------------------------------- distance */

/* Squared Euclidean distance of base row `row` to query `q`, as a double.
 * For u8 and i8 the sum is formed in int64 and is exact; for f32 every
 * component is widened to double before subtracting. */
static double orc_dist(const void *base, int64_t row, int32_t d, int32_t dtype,
                       const void *q) {
  if (dtype == ORC_U8) {
    const uint8_t *a = (const uint8_t *)base + row * (int64_t)d;
    const uint8_t *b = (const uint8_t *)q;
    int64_t s = 0;
    for (int32_t j = 0; j < d; j++) {
      int64_t t = (int64_t)a[j] - (int64_t)b[j];
      s += t * t;
    }
    return (double)s;
  }
  if (dtype == ORC_I8) {
    const int8_t *a = (const int8_t *)base + row * (int64_t)d;
    const int8_t *b = (const int8_t *)q;
    int64_t s = 0;
    for (int32_t j = 0; j < d; j++) {
      int64_t t = (int64_t)a[j] - (int64_t)b[j];
      s += t * t;
    }
    return (double)s;
  }
  {
    const float *a = (const float *)base + row * (int64_t)d;
    const float *b = (const float *)q;
    double s = 0.0;
    for (int32_t j = 0; j < d; j++) {
      double t = (double)a[j] - (double)b[j];
      s += t * t;
    }
    return s;
  }
}

static size_t orc_elem_bytes(int32_t dtype) { return dtype == ORC_F32 ? 4 : 1; }

/* Exported so tests can pin the distance against a library routine. */
int oracle_distances(const void *base, int64_t n, int32_t d, int32_t dtype,
                     const void *query, double *out) {
  if (!base || !query || !out || n < 0 || d < 1 ||
      (dtype != ORC_U8 && dtype != ORC_I8 && dtype != ORC_F32))
    return ORC_EINVAL;
  for (int64_t i = 0; i < n; i++) out[i] = orc_dist(base, i, d, dtype, query);
  return 0;
}

/* ------------------------------------------------------ product quantisation */

/* Codebooks: M subspaces, subspace m holding dimensions [m*dsub, (m+1)*dsub)
 * with dsub = d / M; 256 centroids of dsub floats each, laid out
 * codebooks[(m * 256 + c) * dsub + j].
 *
 * All PQ arithmetic is fp32 in one fixed order (the paper does not state a
 * precision; a code or a candidate's place in the list is an integer decision
 * that the GPU must take identically):
 *   sub-distance(x, centroid) = acc after acc = fmaf(t, t, acc), t = x_j - c_j,
 *                               for j = 0 .. dsub-1 in order, from acc = 0,
 *                               vector components converted to float (exact
 *                               for u8 and i8)
 *   code of x, subspace m     = the centroid with the smallest sub-distance,
 *                               the lowest index among equals
 *   table of a query          = tab[m * 256 + c] = sub-distance(q_m, centroid c)
 *   PQ distance of a code     = sum over m = 0 .. M-1 in order of
 *                               tab[m * 256 + code_m], in float, from 0   */

#define ORC_KSUB 256

static void orc_row_float(const void *base, int64_t row, int32_t d, int32_t dtype, float *out) {
  for (int32_t j = 0; j < d; j++) {
    if (dtype == ORC_U8)
      out[j] = (float)((const uint8_t *)base)[row * (int64_t)d + j];
    else if (dtype == ORC_I8)
      out[j] = (float)((const int8_t *)base)[row * (int64_t)d + j];
    else
      out[j] = ((const float *)base)[row * (int64_t)d + j];
  }
}

static float orc_pq_sub(const float *x, const float *c, int32_t dsub) {
  float acc = 0.0f;
  for (int32_t j = 0; j < dsub; j++) {
    const float t = x[j] - c[j];
    acc = fmaf(t, t, acc);
  }
  return acc;
}

static int orc_pq_check(int32_t d, int32_t M) { return M >= 1 && M <= d && d % M == 0; }

/* Codes of n base rows: codes[i * M + m]. */
int oracle_pq_encode(const void *base, int64_t n, int32_t d, int32_t dtype,
                     const float *codebooks, int32_t M, uint8_t *codes) {
  if (!base || !codebooks || !codes || n < 0 || !orc_pq_check(d, M) ||
      (dtype != ORC_U8 && dtype != ORC_I8 && dtype != ORC_F32))
    return ORC_EINVAL;
  const int32_t dsub = d / M;
  float *x = (float *)malloc(sizeof(float) * (size_t)d);
  if (!x) return ORC_ENOMEM;
  for (int64_t i = 0; i < n; i++) {
    orc_row_float(base, i, d, dtype, x);
    for (int32_t m = 0; m < M; m++) {
      int32_t best = 0;
      float bd = 0.0f;
      for (int32_t c = 0; c < ORC_KSUB; c++) {
        const float s = orc_pq_sub(x + m * dsub, codebooks + ((int64_t)m * ORC_KSUB + c) * dsub, dsub);
        if (c == 0 || s < bd) {
          bd = s;
          best = c;
        }
      }
      codes[i * M + m] = (uint8_t)best;
    }
  }
  free(x);
  return 0;
}

/* Distance table of one query (d elements of `dtype`): tab[m * 256 + c]. */
int oracle_pq_table(const void *query, int32_t d, int32_t dtype, const float *codebooks,
                    int32_t M, float *tab) {
  if (!query || !codebooks || !tab || !orc_pq_check(d, M) ||
      (dtype != ORC_U8 && dtype != ORC_I8 && dtype != ORC_F32))
    return ORC_EINVAL;
  const int32_t dsub = d / M;
  float *x = (float *)malloc(sizeof(float) * (size_t)d);
  if (!x) return ORC_ENOMEM;
  orc_row_float(query, 0, d, dtype, x);
  for (int32_t m = 0; m < M; m++)
    for (int32_t c = 0; c < ORC_KSUB; c++)
      tab[m * ORC_KSUB + c] =
          orc_pq_sub(x + m * dsub, codebooks + ((int64_t)m * ORC_KSUB + c) * dsub, dsub);
  free(x);
  return 0;
}

static float orc_pq_dist(const float *tab, const uint8_t *code, int32_t M) {
  float s = 0.0f;
  for (int32_t m = 0; m < M; m++) s += tab[m * ORC_KSUB + code[m]];
  return s;
}

/* ------------------------------------------------------------- keys, lists */

typedef struct {
  double dist;
  int32_t id;
  int32_t expanded;
} orc_entry;

/* Lexicographic (distance, id) order. */
static int orc_cmp(const void *pa, const void *pb) {
  const orc_entry *a = (const orc_entry *)pa, *b = (const orc_entry *)pb;
  if (a->dist < b->dist) return -1;
  if (a->dist > b->dist) return 1;
  if (a->id < b->id) return -1;
  if (a->id > b->id) return 1;
  return 0;
}

/* ------------------------------------------------------------ threads pool */

typedef struct {
  int64_t next;
  pthread_mutex_t mu;
} orc_counter;

static int64_t orc_take(orc_counter *c) {
  pthread_mutex_lock(&c->mu);
  int64_t i = c->next++;
  pthread_mutex_unlock(&c->mu);
  return i;
}

/* ------------------------------------------------------------ brute force */

typedef struct {
  const void *base;
  int64_t n;
  int32_t d, dtype;
  const void *queries;
  int64_t nq;
  int32_t k;
  int32_t *ids;
  double *dists;
  orc_counter *ctr;
  int err;
} orc_bf_job;

static void *orc_bf_worker(void *arg) {
  orc_bf_job *J = (orc_bf_job *)arg;
  orc_entry *all = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(J->n > 0 ? J->n : 1));
  if (!all) {
    J->err = ORC_ENOMEM;
    return NULL;
  }
  size_t qbytes = (size_t)J->d * orc_elem_bytes(J->dtype);
  for (;;) {
    int64_t qi = orc_take(J->ctr);
    if (qi >= J->nq) break;
    const void *q = (const char *)J->queries + qi * qbytes;
    for (int64_t i = 0; i < J->n; i++) {
      all[i].dist = orc_dist(J->base, i, J->d, J->dtype, q);
      all[i].id = (int32_t)i;
      all[i].expanded = 0;
    }
    qsort(all, (size_t)J->n, sizeof(orc_entry), orc_cmp);
    for (int32_t j = 0; j < J->k; j++) {
      if (j < J->n) {
        J->ids[qi * J->k + j] = all[j].id;
        J->dists[qi * J->k + j] = all[j].dist;
      } else {
        J->ids[qi * J->k + j] = -1;
        J->dists[qi * J->k + j] = INFINITY;
      }
    }
  }
  free(all);
  return NULL;
}

static int orc_run_threads(void *(*fn)(void *), void *jobs, size_t job_size,
                           int32_t threads) {
  if (threads < 1) threads = 1;
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
  if (!th) return ORC_ENOMEM;
  int started = 0;
  for (int32_t t = 0; t < threads; t++) {
    if (pthread_create(&th[t], NULL, fn, (char *)jobs + job_size * (size_t)t) != 0) break;
    started++;
  }
  for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
  free(th);
  return started > 0 ? 0 : ORC_ENOMEM;
}

/* Exact top-k by full scan (the definition of k-nearest neighbours). */
int oracle_bruteforce(const void *base, int64_t n, int32_t d, int32_t dtype,
                      const void *queries, int64_t nq, int32_t k, int32_t threads,
                      int32_t *ids, double *dists) {
  if (!base || (!queries && nq > 0) || (nq > 0 && (!ids || !dists)) || n < 0 ||
      nq < 0 || d < 1 || k < 1 ||
      (dtype != ORC_U8 && dtype != ORC_I8 && dtype != ORC_F32))
    return ORC_EINVAL;
  if (nq == 0) return 0;
  if (threads < 1) threads = 1;
  orc_counter ctr = {0, PTHREAD_MUTEX_INITIALIZER};
  orc_bf_job *jobs = (orc_bf_job *)calloc((size_t)threads, sizeof(orc_bf_job));
  if (!jobs) return ORC_ENOMEM;
  for (int32_t t = 0; t < threads; t++) {
    orc_bf_job j = {base, n, d, dtype, queries, nq, k, ids, dists, &ctr, 0};
    jobs[t] = j;
  }
  int rc = orc_run_threads(orc_bf_worker, jobs, sizeof(orc_bf_job), threads);
  for (int32_t t = 0; t < threads && rc == 0; t++)
    if (jobs[t].err) rc = jobs[t].err;
  free(jobs);
  return rc;
}

/* ----------------------------------------------------------------- search */

typedef struct {
  const void *base;
  int64_t n;
  int32_t d, dtype;
  const int32_t *adj;
  int32_t adj_stride, entry;
  const void *queries;
  int64_t nq;
  int32_t k, L, R, delay, beam;
  int32_t *ids;
  double *dists;
  uint32_t *steps;
  int32_t *trace;   /* nq x trace_cap selected ids, -1 padded (optional) */
  double *theta;    /* nq x trace_cap: L-th distance after each processing */
  int32_t trace_cap;
  orc_counter *ctr;
  int err;
  /* compressed navigation (optional): codes n x pq_m, codebooks */
  const uint8_t *pq_codes;
  const float *pq_cb;
  int32_t pq_m;
} orc_search_job;

/* Work buffers of one worker thread. */
typedef struct {
  uint8_t *visited;
  orc_entry *cand, *merged, *res;
  int32_t *fifo;
  float *tab;
} orc_work;

/* Navigation distance of node x: exact, or the PQ distance of its code. */
static double orc_nav_dist(const orc_search_job *J, const orc_work *w, const void *q, int32_t x) {
  if (J->pq_codes) return (double)orc_pq_dist(w->tab, J->pq_codes + (int64_t)x * J->pq_m, J->pq_m);
  return orc_dist(J->base, x, J->d, J->dtype, q);
}

/* One query of the search.  Work buffers are owned by the caller. */
static void orc_search_one(const orc_search_job *J, int64_t qi, const orc_work *w) {
  uint8_t *visited = w->visited;
  orc_entry *cand = w->cand, *merged = w->merged, *res = w->res;
  int32_t *fifo = w->fifo;
  const size_t qbytes = (size_t)J->d * orc_elem_bytes(J->dtype);
  const void *q = (const char *)J->queries + qi * qbytes;
  const int32_t L = J->L, W = J->beam;
  const int32_t fifo_cap = (J->delay + 1) * W + W;
  int32_t *tr = J->trace ? J->trace + qi * J->trace_cap : NULL;
  double *th = J->theta ? J->theta + qi * J->trace_cap : NULL;
  if (tr)
    for (int32_t i = 0; i < J->trace_cap; i++) tr[i] = -1;
  if (th)
    for (int32_t i = 0; i < J->trace_cap; i++) th[i] = NAN;

  memset(visited, 0, (size_t)J->n);
  if (J->pq_codes) oracle_pq_table(q, J->d, J->dtype, J->pq_cb, J->pq_m, w->tab);
  int64_t nres = 0; /* compressed navigation: exact distances of expanded nodes */
  /* Init: the candidate list holds the entry node only; it is visited. */
  int32_t nc = 1;
  cand[0].dist = orc_nav_dist(J, w, q, J->entry);
  cand[0].id = J->entry;
  cand[0].expanded = 0;
  visited[J->entry] = 1;

  int32_t f_head = 0, f_len = 0; /* circular FIFO of in-flight node ids */
  uint32_t steps = 0, processed = 0;

  for (;;) {
    /* Select: up to W first unexpanded entries, in list order. */
    int32_t nsel = 0;
    for (int32_t i = 0; i < nc && nsel < W; i++) {
      if (cand[i].expanded) continue;
      cand[i].expanded = 1;
      fifo[(f_head + f_len) % fifo_cap] = cand[i].id;
      f_len++;
      if (tr && steps < (uint32_t)J->trace_cap) tr[steps] = cand[i].id;
      steps++;
      nsel++;
    }
    if (nsel == 0 && f_len == 0) break; /* nothing left to select or finish */

    /* Process: while more than delay*W nodes are in flight; when nothing new
     * was selected, drain up to W of the oldest in-flight nodes. */
    int32_t to_process = 0;
    if (f_len > J->delay * W) to_process = f_len - J->delay * W;
    if (nsel == 0 && to_process == 0) to_process = f_len < W ? f_len : W;

    for (int32_t p = 0; p < to_process; p++) {
      int32_t u = fifo[f_head];
      f_head = (f_head + 1) % fifo_cap;
      f_len--;
      if (J->pq_codes) { /* u's record holds its full vector: exact distance */
        res[nres].dist = orc_dist(J->base, u, J->d, J->dtype, q);
        res[nres].id = u;
        res[nres].expanded = 1;
        nres++;
      }
      /* Neighbours: the first R ids of u's list that are not yet visited. */
      int32_t m = 0;
      for (int32_t i = 0; i < nc; i++) merged[m++] = cand[i];
      const int32_t *nb = J->adj + (int64_t)u * J->adj_stride;
      for (int32_t j = 0; j < J->R; j++) {
        int32_t x = nb[j];
        if (x < 0 || (int64_t)x >= J->n) continue; /* padding slot */
        if (visited[x]) continue;
        visited[x] = 1;
        merged[m].dist = orc_nav_dist(J, w, q, x);
        merged[m].id = x;
        merged[m].expanded = 0;
        m++;
      }
      /* C = first L of sort(C u new). */
      qsort(merged, (size_t)m, sizeof(orc_entry), orc_cmp);
      nc = m < L ? m : L;
      for (int32_t i = 0; i < nc; i++) cand[i] = merged[i];
      if (th && processed < (uint32_t)J->trace_cap)
        th[processed] = (nc == L) ? cand[L - 1].dist : INFINITY;
      processed++;
    }
  }

  /* The answer: the first k of the list, or with compressed navigation the
   * first k of the expanded nodes by exact distance. */
  const orc_entry *out = cand;
  int64_t nout = nc;
  if (J->pq_codes) {
    qsort(res, (size_t)nres, sizeof(orc_entry), orc_cmp);
    out = res;
    nout = nres;
  }
  for (int32_t j = 0; j < J->k; j++) {
    if (j < nout) {
      J->ids[qi * J->k + j] = out[j].id;
      J->dists[qi * J->k + j] = out[j].dist;
    } else {
      J->ids[qi * J->k + j] = -1;
      J->dists[qi * J->k + j] = INFINITY;
    }
  }
  if (J->steps) J->steps[qi] = steps;
}

static void *orc_search_worker(void *arg) {
  orc_search_job *J = (orc_search_job *)arg;
  const int32_t W = J->beam;
  orc_work w;
  w.visited = (uint8_t *)malloc((size_t)(J->n > 0 ? J->n : 1));
  w.cand = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)J->L);
  w.merged = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(J->L + J->R + 1));
  w.fifo = (int32_t *)malloc(sizeof(int32_t) * (size_t)((J->delay + 2) * W));
  /* each node is expanded at most once: n result entries suffice */
  w.res = J->pq_codes ? (orc_entry *)malloc(sizeof(orc_entry) * (size_t)J->n) : NULL;
  w.tab = J->pq_codes ? (float *)malloc(sizeof(float) * (size_t)J->pq_m * ORC_KSUB) : NULL;
  if (!w.visited || !w.cand || !w.merged || !w.fifo || (J->pq_codes && (!w.res || !w.tab))) {
    J->err = ORC_ENOMEM;
  } else {
    for (;;) {
      int64_t qi = orc_take(J->ctr);
      if (qi >= J->nq) break;
      orc_search_one(J, qi, &w);
    }
  }
  free(w.visited);
  free(w.cand);
  free(w.merged);
  free(w.fifo);
  free(w.res);
  free(w.tab);
  return NULL;
}

/*
 * oracle_search: batched best-first search, strict (delay = 0) or relaxed.
 *   base      n x d row-major vectors (u8, i8 or f32 by dtype)
 *   adj       n x adj_stride int32 neighbour ids; the first R of each row are
 *             used; ids outside [0, n) are padding and ignored
 *   entry     entrance node id
 *   queries   nq x d, same dtype as base
 *   k, L      results per query and candidate-list size (1 <= k <= L)
 *   R         neighbours used per expansion (1 <= R <= adj_stride)
 *   delay     staleness (>= 0); beam = nodes selected per iteration (>= 1)
 *   ids/dists nq x k outputs, padded with -1 / +inf
 *   steps     nq expansions (selections) per query, optional
 *   trace     nq x trace_cap selected ids in order, optional
 *   theta     nq x trace_cap, the L-th distance after each processed node
 *             (+inf while fewer than L candidates), optional
 * Returns 0, -22 on invalid arguments, -12 on allocation failure.
 */
static int orc_search_all(const void *base, int64_t n, int32_t d, int32_t dtype,
                          const int32_t *adj, int32_t adj_stride, int32_t entry,
                          const void *queries, int64_t nq, int32_t k, int32_t L, int32_t R,
                          int32_t delay, int32_t beam, int32_t threads, int32_t *ids,
                          double *dists, uint32_t *steps, int32_t *trace, double *theta,
                          int32_t trace_cap, const uint8_t *pq_codes, const float *pq_cb,
                          int32_t pq_m) {
  if (!base || !adj || n < 1 || d < 1 || nq < 0 ||
      (dtype != ORC_U8 && dtype != ORC_I8 && dtype != ORC_F32))
    return ORC_EINVAL;
  if (nq > 0 && (!queries || !ids || !dists)) return ORC_EINVAL;
  if (k < 1 || L < k || R < 1 || R > adj_stride || delay < 0 || beam < 1)
    return ORC_EINVAL;
  if (entry < 0 || (int64_t)entry >= n) return ORC_EINVAL;
  if ((trace || theta) && trace_cap < 1) return ORC_EINVAL;
  if (nq == 0) return 0;
  if (threads < 1) threads = 1;
  orc_counter ctr = {0, PTHREAD_MUTEX_INITIALIZER};
  orc_search_job *jobs = (orc_search_job *)calloc((size_t)threads, sizeof(orc_search_job));
  if (!jobs) return ORC_ENOMEM;
  for (int32_t t = 0; t < threads; t++) {
    orc_search_job j = {base,  n,     d,     dtype, adj,   adj_stride, entry,
                        queries, nq,  k,     L,     R,     delay,      beam,
                        ids,   dists, steps, trace, theta, trace_cap,  &ctr,
                        0,     pq_codes, pq_cb, pq_m};
    jobs[t] = j;
  }
  int rc = orc_run_threads(orc_search_worker, jobs, sizeof(orc_search_job), threads);
  for (int32_t t = 0; t < threads && rc == 0; t++)
    if (jobs[t].err) rc = jobs[t].err;
  free(jobs);
  return rc;
}

int oracle_search(const void *base, int64_t n, int32_t d, int32_t dtype,
                  const int32_t *adj, int32_t adj_stride, int32_t entry,
                  const void *queries, int64_t nq, int32_t k, int32_t L, int32_t R,
                  int32_t delay, int32_t beam, int32_t threads, int32_t *ids,
                  double *dists, uint32_t *steps, int32_t *trace, double *theta,
                  int32_t trace_cap) {
  return orc_search_all(base, n, d, dtype, adj, adj_stride, entry, queries, nq, k, L, R, delay,
                        beam, threads, ids, dists, steps, trace, theta, trace_cap, NULL, NULL, 0);
}

/*
 * oracle_search_pq: the same search with compressed navigation.  The base is
 * encoded with `codebooks` (M subspaces, see oracle_pq_encode); the list is
 * ordered by PQ distance (`theta` then holds the L-th PQ distance); ids and
 * dists are the first k of the expanded nodes by exact distance (float64,
 * exact for u8/i8), padded with -1 / +inf.  Other arguments as oracle_search.
 */
/* Rows [i0, i1) of the base encoded by one thread (oracle_pq_encode on a slice). */
typedef struct {
  const void *base;
  int64_t i0, i1;
  int32_t d, dtype, M;
  const float *cb;
  uint8_t *codes;
  int err;
} orc_enc_job;

static void *orc_enc_worker(void *arg) {
  orc_enc_job *J = (orc_enc_job *)arg;
  const size_t row = (size_t)J->d * orc_elem_bytes(J->dtype);
  if (J->i1 > J->i0)
    J->err = oracle_pq_encode((const char *)J->base + (size_t)J->i0 * row, J->i1 - J->i0, J->d,
                              J->dtype, J->cb, J->M, J->codes + J->i0 * J->M);
  return NULL;
}

static int orc_pq_encode_threads(const void *base, int64_t n, int32_t d, int32_t dtype,
                                 const float *cb, int32_t M, uint8_t *codes, int32_t threads) {
  if (threads < 1) threads = 1;
  orc_enc_job *jobs = (orc_enc_job *)calloc((size_t)threads, sizeof(orc_enc_job));
  if (!jobs) return ORC_ENOMEM;
  for (int32_t t = 0; t < threads; t++) {
    orc_enc_job j = {base, n * t / threads, n * (t + 1) / threads, d, dtype, M, cb, codes, 0};
    jobs[t] = j;
  }
  int rc = orc_run_threads(orc_enc_worker, jobs, sizeof(orc_enc_job), threads);
  for (int32_t t = 0; t < threads && rc == 0; t++)
    if (jobs[t].err) rc = jobs[t].err;
  free(jobs);
  return rc;
}

int oracle_search_pq(const void *base, int64_t n, int32_t d, int32_t dtype,
                     const int32_t *adj, int32_t adj_stride, int32_t entry,
                     const void *queries, int64_t nq, int32_t k, int32_t L, int32_t R,
                     int32_t delay, int32_t beam, int32_t threads, int32_t *ids,
                     double *dists, uint32_t *steps, int32_t *trace, double *theta,
                     int32_t trace_cap, const float *codebooks, int32_t M) {
  if (!base || !codebooks || n < 1 || !orc_pq_check(d, M)) return ORC_EINVAL;
  uint8_t *codes = (uint8_t *)malloc((size_t)n * (size_t)M);
  if (!codes) return ORC_ENOMEM;
  int rc = orc_pq_encode_threads(base, n, d, dtype, codebooks, M, codes, threads);
  if (rc == 0)
    rc = orc_search_all(base, n, d, dtype, adj, adj_stride, entry, queries, nq, k, L, R, delay,
                        beam, threads, ids, dists, steps, trace, theta, trace_cap, codes,
                        codebooks, M);
  free(codes);
  return rc;
}

/*
 * oracle.c - plain, slow CPU oracle for neighbourhood-based link prediction
 * (IBase and DLH) in FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header, table or constant with the GPU
 * implementation.
 *
 * What is computed (Sahu, "A Fast Parallel Approach for Neighborhood-based
 * Link Prediction by Disregarding Large Hubs"):
 *   Gamma_v is the neighbour set of v in the observed graph, d_v = |Gamma_v|.
 *   An intermediate b is explored iff d_b <= L (Section 4.2.1, the hub limit;
 *   IBase is L = infinity, Section 4.4).  For a != c,
 *     h(a,c) = |{ b in Gamma_a n Gamma_c : d_b <= L }|
 *   Candidates are unordered pairs a < c, c not in Gamma_a, h >= 1
 *   (Sections 4.1.1, 4.1.2, 4.1.4).  Scores are the nine measures of
 *   Section 3.1 (equations CN ... RA), with the union of Section 4.1.2,
 *   |Gamma_a u Gamma_c| = d_a + d_c - h, and AA/RA summed over the
 *   common (explored) intermediates, natural log.
 *   A prediction keeps scores strictly above S_th (Algorithm 1, scoring
 *   phase) and the top N_P by (fp32 score desc, a asc, c asc).
 *
 * Two independent routes:
 *   O0  oracle_bruteforce / oracle_pair: the definition written out, by merge
 *       intersection of two sorted neighbour lists, for every pair (Section
 *       3.3, the baseline approach).
 *   O1  oracle_source / oracle_predict / oracle_query / oracle_fingerprint:
 *       the paper's algorithm (Section 4.1, Algorithm 1): per source a, a
 *       depth-2 traversal that accumulates into a collision-free per-thread
 *       table (a values vector of size |V|, a keys vector and a key count),
 *       skipping c <= a and hub intermediates, then clearing first-order
 *       neighbours, then scoring; per-thread bounded min-heaps of size N_P
 *       followed by a sort and max-heap merge.  Ties are broken by the total
 *       order above so the result is deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { M_CN = 0, M_JC, M_SI, M_SC, M_HP, M_HD, M_LHN, M_AA, M_RA, M_COUNT };

/* ---------------------------------------------------------------------- */
/* Scores (Section 3.1, equations for CN, JC, SI, SC, HP, HD, LHN, AA, RA) */
/* ---------------------------------------------------------------------- */

/* weight contributed by one explored common neighbour b (AA / RA) */
double oracle_weight(int m, int64_t db) {
  if (m == M_AA) return db > 1 ? 1.0 / log((double)db) : 0.0;
  if (m == M_RA) return db > 0 ? 1.0 / (double)db : 0.0;
  return 1.0;
}

double oracle_score(int m, int64_t h, double w, int64_t da, int64_t dc) {
  double H = (double)h, A = (double)da, C = (double)dc;
  switch (m) {
    case M_CN: return H;
    case M_JC: return H / (double)(da + dc - h);
    case M_SI: return H / (double)(da + dc);
    case M_SC: return H / sqrt(A * C);
    case M_HP: return H / (double)(da < dc ? da : dc);
    case M_HD: return H / (double)(da > dc ? da : dc);
    case M_LHN: return H / (A * C);
    case M_AA: return w;
    case M_RA: return w;
    default: return 0.0;
  }
}

static inline int64_t deg_of(const int64_t *off, int64_t v) { return off[v + 1] - off[v]; }
static inline int explored(const int64_t *off, int64_t b, int64_t L) { return deg_of(off, b) <= L; }

/* ---------------------------------------------------------------------- */
/* O0: the definition, pair by pair                                        */
/* ---------------------------------------------------------------------- */

static int adjacent(const int64_t *off, const int32_t *idx, int64_t a, int64_t c) {
  int64_t lo = off[a], hi = off[a + 1];
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (idx[mid] < c) lo = mid + 1; else hi = mid;
  }
  return lo < off[a + 1] && idx[lo] == c;
}

/* h and the AA/RA weight sum for one pair, by merging two sorted lists */
static void pair_counts(const int64_t *off, const int32_t *idx, int64_t L, int m,
                        int64_t a, int64_t c, int64_t *h, double *w) {
  int64_t i = off[a], ie = off[a + 1], j = off[c], je = off[c + 1];
  int64_t cnt = 0;
  double sum = 0.0;
  while (i < ie && j < je) {
    if (idx[i] < idx[j]) i++;
    else if (idx[i] > idx[j]) j++;
    else {
      int64_t b = idx[i];
      if (explored(off, b, L)) { cnt++; sum += oracle_weight(m, deg_of(off, b)); }
      i++; j++;
    }
  }
  *h = cnt;
  *w = sum;
}

static int get_threads(int nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* One pair: returns 1 and fills h / score if (a, c) is a candidate. */
int oracle_pair(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m,
                int64_t a, int64_t c, int64_t *h_out, double *s_out) {
  (void)n;
  int64_t h = 0;
  double w = 0;
  *h_out = 0;
  *s_out = 0;
  if (a == c || adjacent(off, idx, a, c)) return 0;
  pair_counts(off, idx, L, m, a, c, &h, &w);
  *h_out = h;
  if (h == 0) return 0;
  *s_out = oracle_score(m, h, w, deg_of(off, a), deg_of(off, c));
  return 1;
}

/* oracle_pair over a list of unordered pairs (a[i], c[i]); ok[i] = 1 for a
 * candidate, with its h and FP64 score.  Used to check a listed pair that
 * another route reported without re-running a whole prediction. */
void oracle_pairs(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m,
                  const int32_t *a, const int32_t *c, int64_t np, int nthreads,
                  int8_t *ok, int64_t *h_out, double *s_out) {
  int T = get_threads(nthreads);
#pragma omp parallel for num_threads(T) schedule(dynamic, 64)
  for (int64_t i = 0; i < np; i++) {
    int valid = a[i] >= 0 && a[i] < n && c[i] >= 0 && c[i] < n;
    h_out[i] = 0;
    s_out[i] = 0.0;
    ok[i] = valid ? (int8_t)oracle_pair(n, off, idx, L, m, a[i], c[i], &h_out[i], &s_out[i]) : 0;
  }
}

/* Every candidate pair a < c; returns the total count, writes up to cap. */
int64_t oracle_bruteforce(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m,
                          int32_t *out_a, int32_t *out_c, int64_t *out_h, double *out_s,
                          int64_t cap) {
  int64_t t = 0;
  for (int64_t a = 0; a < n; a++) {
    for (int64_t c = a + 1; c < n; c++) {
      int64_t h;
      double s;
      if (!oracle_pair(n, off, idx, L, m, a, c, &h, &s)) continue;
      if (t < cap) {
        out_a[t] = (int32_t)a;
        out_c[t] = (int32_t)c;
        out_h[t] = h;
        out_s[t] = s;
      }
      t++;
    }
  }
  return t;
}

/* ---------------------------------------------------------------------- */
/* O1: the paper's two-hop algorithm                                       */
/* ---------------------------------------------------------------------- */

/* collision-free per-thread table: a values vector of size |V| (count and
 * weight), a keys vector and a key count (Section 4.1.3). */
typedef struct {
  int64_t *cnt;
  double *w;
  int32_t *keys;
  int64_t nkeys;
  uint8_t *seen; /* seen[c] != 0 when c is already a key of the current source */
} table_t;

static int table_init(table_t *t, int64_t n) {
  size_t N = (size_t)(n > 0 ? n : 1);
  t->cnt = (int64_t *)calloc(N, sizeof(int64_t));
  t->w = (double *)calloc(N, sizeof(double));
  t->keys = (int32_t *)malloc(N * sizeof(int32_t));
  t->seen = (uint8_t *)calloc(N, sizeof(uint8_t));
  t->nkeys = 0;
  return t->cnt && t->w && t->keys && t->seen;
}
static void table_free(table_t *t) {
  free(t->cnt); free(t->w); free(t->keys); free(t->seen);
}

/* mode 0: prediction orientation (skip c <= a, Algorithm 1 scanEdges);
 * mode 1: recommendation for one vertex (skip only c == a). */
static void scan_edges(table_t *t, const int64_t *off, const int32_t *idx, int m,
                       int64_t a, int64_t b, int mode) {
  double wb = oracle_weight(m, deg_of(off, b));
  for (int64_t e = off[b]; e < off[b + 1]; e++) {
    int64_t c = idx[e];
    if (mode == 0 ? c <= a : c == a) continue;
    if (!t->seen[c]) { t->seen[c] = 1; t->keys[t->nkeys++] = (int32_t)c; }
    t->cnt[c] += 1;
    t->w[c] += wb;
  }
}

/* Fill the table for source a: traversal, hub filter, first-order clearing. */
static void fill_source(table_t *t, const int64_t *off, const int32_t *idx, int64_t L, int m,
                        int64_t a, int mode) {
  t->nkeys = 0;
  for (int64_t e = off[a]; e < off[a + 1]; e++) {
    int64_t b = idx[e];
    if (explored(off, b, L)) scan_edges(t, off, idx, m, a, b, mode);
  }
  /* first-order neighbours are never candidates (Section 4.1.4) */
  for (int64_t e = off[a]; e < off[a + 1]; e++) {
    int64_t b = idx[e];
    t->cnt[b] = 0;
    t->w[b] = 0.0;
  }
}

static void reset_keys(table_t *t) {
  for (int64_t i = 0; i < t->nkeys; i++) {
    int32_t c = t->keys[i];
    t->cnt[c] = 0;
    t->w[c] = 0.0;
    t->seen[c] = 0;
  }
  t->nkeys = 0;
}

/* Per-source candidate list (c, h, score), in key-insertion order. */
int64_t oracle_source(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m,
                      int64_t a, int mode, int32_t *out_c, int64_t *out_h, double *out_s,
                      int64_t cap) {
  table_t t;
  if (!table_init(&t, n)) { table_free(&t); return -1; }
  fill_source(&t, off, idx, L, m, a, mode);
  int64_t r = 0;
  for (int64_t i = 0; i < t.nkeys; i++) {
    int64_t c = t.keys[i];
    if (t.cnt[c] == 0) continue;
    if (r < cap) {
      out_c[r] = (int32_t)c;
      out_h[r] = t.cnt[c];
      out_s[r] = oracle_score(m, t.cnt[c], t.w[c], deg_of(off, a), deg_of(off, c));
    }
    r++;
  }
  table_free(&t);
  return r;
}

/* ----- prediction lists: bounded min-heaps under the total order ------- */

typedef struct {
  float s32;
  int32_t a, c;
  double s64;
} pred_t;

/* x ranks before y */
static inline int better(const pred_t *x, const pred_t *y) {
  if (x->s32 != y->s32) return x->s32 > y->s32;
  if (x->a != y->a) return x->a < y->a;
  return x->c < y->c;
}

static void sift_down_min(pred_t *h, int64_t n, int64_t i) {
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, w = i;
    if (l < n && better(&h[w], &h[l])) w = l;
    if (r < n && better(&h[w], &h[r])) w = r;
    if (w == i) return;
    pred_t t = h[i]; h[i] = h[w]; h[w] = t;
    i = w;
  }
}

typedef struct {
  pred_t *v;
  int64_t size, cap;
  int heaped;
} plist_t;

/* Algorithm 1: push until N_P entries, then keep a min-heap and replace the
 * worst entry when a better one arrives. */
static void plist_add(plist_t *p, pred_t x) {
  if (p->cap == 0) return;
  if (p->size < p->cap) {
    p->v[p->size++] = x;
    if (p->size == p->cap) {
      for (int64_t i = p->size / 2 - 1; i >= 0; i--) sift_down_min(p->v, p->size, i);
      p->heaped = 1;
    }
  } else if (better(&x, &p->v[0])) {
    p->v[0] = x;
    sift_down_min(p->v, p->size, 0);
  }
}

static int cmp_pred_desc(const void *x, const void *y) {
  const pred_t *a = (const pred_t *)x, *b = (const pred_t *)y;
  if (better(a, b)) return -1;
  if (better(b, a)) return 1;
  return 0;
}

/*
 * Whole-graph prediction.  Returns k' = min(k, |candidates above S_th|) and
 * writes the list in order (fp32 score desc, a asc, c asc); -1 on allocation
 * failure.
 */
int64_t oracle_predict_sources(int64_t n, const int64_t *off, const int32_t *idx, int64_t L,
                               int m, int64_t k, float s_th, int nthreads, const int32_t *sources,
                               int64_t ns, int32_t *out_a, int32_t *out_c, float *out_s32,
                               double *out_s64);

int64_t oracle_predict(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m,
                       int64_t k, float s_th, int nthreads, int32_t *out_a, int32_t *out_c,
                       float *out_s32, double *out_s64) {
  return oracle_predict_sources(n, off, idx, L, m, k, s_th, nthreads, NULL, n, out_a, out_c,
                                out_s32, out_s64);
}

/* The same restricted to the sources listed (all vertices when sources is
 * NULL): the candidates owned by those sources, top k of them. */
int64_t oracle_predict_sources(int64_t n, const int64_t *off, const int32_t *idx, int64_t L,
                               int m, int64_t k, float s_th, int nthreads, const int32_t *sources,
                               int64_t ns, int32_t *out_a, int32_t *out_c, float *out_s32,
                               double *out_s64) {
  int T = get_threads(nthreads);
  plist_t *P = (plist_t *)calloc((size_t)T, sizeof(plist_t));
  int failed = 0;
  for (int t = 0; t < T; t++) {
    P[t].cap = k;
    P[t].v = (pred_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(pred_t));
    if (!P[t].v) failed = 1;
  }
  if (!failed) {
    /* scoring phase: vertices in parallel, dynamic schedule of 2048 (Section 4.1.7) */
#pragma omp parallel num_threads(T)
    {
#ifdef _OPENMP
      int tid = omp_get_thread_num();
#else
      int tid = 0;
#endif
      table_t tb;
      if (!table_init(&tb, n)) {
#pragma omp atomic write
        failed = 1;
      } else {
#pragma omp for schedule(dynamic, 2048)
        for (int64_t i = 0; i < ns; i++) {
          const int64_t a = sources ? sources[i] : i;
          fill_source(&tb, off, idx, L, m, a, 0);
          for (int64_t i = 0; i < tb.nkeys; i++) {
            int64_t c = tb.keys[i];
            if (tb.cnt[c] == 0) continue;
            double s = oracle_score(m, tb.cnt[c], tb.w[c], deg_of(off, a), deg_of(off, c));
            float s32 = (float)s;
            if (!(s32 > s_th)) continue;
            pred_t x = {s32, (int32_t)a, (int32_t)c, s};
            plist_add(&P[tid], x);
          }
          reset_keys(&tb);
        }
      }
      table_free(&tb);
    }
  }
  int64_t r = 0;
  if (!failed) {
    /* merging phase: sort every per-thread list, then a max-heap merge */
    for (int t = 0; t < T; t++) qsort(P[t].v, (size_t)P[t].size, sizeof(pred_t), cmp_pred_desc);
    int64_t *head = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    while (r < k) {
      int best = -1;
      for (int t = 0; t < T; t++) {
        if (head[t] >= P[t].size) continue;
        if (best < 0 || better(&P[t].v[head[t]], &P[best].v[head[best]])) best = t;
      }
      if (best < 0) break;
      pred_t x = P[best].v[head[best]++];
      out_a[r] = x.a;
      out_c[r] = x.c;
      out_s32[r] = x.s32;
      out_s64[r] = x.s64;
      r++;
    }
    free(head);
  }
  for (int t = 0; t < T; t++) free(P[t].v);
  free(P);
  return failed ? -1 : r;
}

/*
 * Recommendation for each vertex in src[0..ns): its candidates c != s,
 * c not in Gamma_s, h >= 1, score > s_th, top kq by (fp32 score desc, c asc).
 * Row i of out_c / out_s32 / out_s64 holds out_cnt[i] entries.
 */
int oracle_query(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m,
                 const int32_t *src, int64_t ns, int32_t kq, float s_th, int nthreads,
                 int32_t *out_c, float *out_s32, double *out_s64, int32_t *out_cnt) {
  int T = get_threads(nthreads);
  int failed = 0;
#pragma omp parallel num_threads(T)
  {
    table_t tb;
    plist_t pl;
    pl.cap = kq;
    pl.v = (pred_t *)malloc((size_t)(kq > 0 ? kq : 1) * sizeof(pred_t));
    if (!table_init(&tb, n) || !pl.v) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < ns; i++) {
        int64_t s = src[i];
        pl.size = 0;
        pl.heaped = 0;
        fill_source(&tb, off, idx, L, m, s, 1);
        for (int64_t j = 0; j < tb.nkeys; j++) {
          int64_t c = tb.keys[j];
          if (tb.cnt[c] == 0) continue;
          double sc = oracle_score(m, tb.cnt[c], tb.w[c], deg_of(off, s), deg_of(off, c));
          float s32 = (float)sc;
          if (!(s32 > s_th)) continue;
          pred_t x = {s32, 0, (int32_t)c, sc};
          plist_add(&pl, x);
        }
        reset_keys(&tb);
        qsort(pl.v, (size_t)pl.size, sizeof(pred_t), cmp_pred_desc);
        for (int64_t j = 0; j < pl.size; j++) {
          out_c[i * kq + j] = pl.v[j].c;
          out_s32[i * kq + j] = pl.v[j].s32;
          out_s64[i * kq + j] = pl.v[j].s64;
        }
        out_cnt[i] = (int32_t)pl.size;
      }
    }
    table_free(&tb);
    free(pl.v);
  }
  return failed ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Order-independent digest of the whole candidate set                     */
/* ---------------------------------------------------------------------- */

/* SplitMix64 finaliser (Steele, Lea, Flood 2014) applied to (a, c, h). */
static inline uint64_t fp_mix(uint64_t a, uint64_t c, uint64_t h) {
  uint64_t z = ((a << 32) | (c & 0xFFFFFFFFULL)) ^ (h * 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* out[0] = |C_L|, out[1] = sum of h, out[2] = sum of fp_mix(a, c, h) (mod 2^64),
 * out[3] = wedges explored with c > a (sum over sources). */
int oracle_fingerprint(int64_t n, const int64_t *off, const int32_t *idx, int64_t L,
                       int nthreads, uint64_t *out) {
  int T = get_threads(nthreads);
  uint64_t cnt = 0, sh = 0, sm = 0, wed = 0;
  int failed = 0;
#pragma omp parallel num_threads(T) reduction(+ : cnt, sh, sm, wed)
  {
    table_t tb;
    if (!table_init(&tb, n)) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 2048)
      for (int64_t a = 0; a < n; a++) {
        fill_source(&tb, off, idx, L, M_CN, a, 0);
        for (int64_t i = 0; i < tb.nkeys; i++) {
          int64_t c = tb.keys[i];
          if (tb.cnt[c] == 0) continue;
          cnt += 1;
          sh += (uint64_t)tb.cnt[c];
          sm += fp_mix((uint64_t)a, (uint64_t)c, (uint64_t)tb.cnt[c]);
        }
        for (int64_t e = off[a]; e < off[a + 1]; e++) {
          int64_t b = idx[e];
          if (!explored(off, b, L)) continue;
          for (int64_t f = off[b]; f < off[b + 1]; f++) wed += (idx[f] > a);
        }
        reset_keys(&tb);
      }
    }
    table_free(&tb);
  }
  out[0] = cnt;
  out[1] = sh;
  out[2] = sm;
  out[3] = wed;
  return failed ? -1 : 0;
}

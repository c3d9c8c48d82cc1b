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
 *       the same sums gathered by intermediate (Sections 4.1 and 4.2): for a
 *       source a, every explored neighbour b adds one (or its AA / RA weight)
 *       to each neighbour c of b, into dense per-thread arrays over the
 *       vertices; neighbours of a are flagged and never candidates.  The k
 *       best under the total order above are kept per thread by sorting and
 *       cutting a bounded buffer, then the threads' sorted lists are merged,
 *       so the result is deterministic.
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
/* O1: accumulation by intermediate (Sections 4.1 and 4.2)                 */
/* ---------------------------------------------------------------------- */

/* h(a, c) counts the explored vertices adjacent to both a and c.  Summed the
 * other way round, each explored neighbour b of a adds one to h(a, c) for
 * every neighbour c of b, so one pass over the explored neighbours of a gives
 * h(a, c), and the AA / RA sum of the weights of those b, for all c at once.
 * The sums of the current source live in dense per-thread arrays indexed by
 * c (a vector of |V| values, as Section 4.1.3 keeps), with a list of the
 * entries touched so that reading and clearing them costs the work done; a
 * flag array marks the neighbours of a, which are never candidates (Section
 * 4.1.4). */
typedef struct {
  int64_t *h;       /* explored common neighbours with the source */
  double *w;        /* sum of their AA / RA weights */
  int32_t *touched; /* entries with h > 0, in order of first touch */
  int64_t ntouched;
  uint8_t *adj_a;   /* 1 at the neighbours of the source */
} sums_t;

static int sums_init(sums_t *t, int64_t n) {
  size_t N = (size_t)(n > 0 ? n : 1);
  t->h = (int64_t *)calloc(N, sizeof(int64_t));
  t->w = (double *)calloc(N, sizeof(double));
  t->touched = (int32_t *)malloc(N * sizeof(int32_t));
  t->adj_a = (uint8_t *)calloc(N, sizeof(uint8_t));
  t->ntouched = 0;
  return t->h && t->w && t->touched && t->adj_a;
}
static void sums_free(sums_t *t) {
  free(t->h); free(t->w); free(t->touched); free(t->adj_a);
}

/* The sums of source a.  mode 0 (prediction): every unordered pair is formed
 * once, by its smaller endpoint, so only c > a is counted (Section 4.1.1);
 * mode 1 (the recommendations of one vertex): every c != a. */
static void sums_of(sums_t *t, const int64_t *off, const int32_t *idx, int64_t L, int m, int64_t a,
                    int mode) {
  t->ntouched = 0;
  for (int64_t e = off[a]; e < off[a + 1]; e++) {
    const int64_t b = idx[e];
    if (!explored(off, b, L)) continue;
    const double wb = oracle_weight(m, deg_of(off, b));
    for (int64_t f = off[b]; f < off[b + 1]; f++) {
      const int64_t c = idx[f];
      if (c == a || (mode == 0 && c < a)) continue;
      if (t->h[c] == 0) t->touched[t->ntouched++] = (int32_t)c;
      t->h[c] += 1;
      t->w[c] += wb;
    }
  }
  for (int64_t e = off[a]; e < off[a + 1]; e++) t->adj_a[idx[e]] = 1;
}

/* c is a candidate of the current source: a common explored neighbour and no edge */
static inline int is_candidate(const sums_t *t, int64_t c) { return t->h[c] > 0 && !t->adj_a[c]; }

static void sums_clear(sums_t *t, const int64_t *off, const int32_t *idx, int64_t a) {
  for (int64_t i = 0; i < t->ntouched; i++) {
    const int32_t c = t->touched[i];
    t->h[c] = 0;
    t->w[c] = 0.0;
  }
  t->ntouched = 0;
  for (int64_t e = off[a]; e < off[a + 1]; e++) t->adj_a[idx[e]] = 0;
}

/* Per-source candidate list (c, h, score), in order of first touch. */
int64_t oracle_source(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m,
                      int64_t a, int mode, int32_t *out_c, int64_t *out_h, double *out_s,
                      int64_t cap) {
  sums_t t;
  if (!sums_init(&t, n)) { sums_free(&t); return -1; }
  sums_of(&t, off, idx, L, m, a, mode);
  int64_t r = 0;
  for (int64_t i = 0; i < t.ntouched; i++) {
    const int64_t c = t.touched[i];
    if (!is_candidate(&t, c)) continue;
    if (r < cap) {
      out_c[r] = (int32_t)c;
      out_h[r] = t.h[c];
      out_s[r] = oracle_score(m, t.h[c], t.w[c], deg_of(off, a), deg_of(off, c));
    }
    r++;
  }
  sums_free(&t);
  return r;
}

/* ----- the k best predictions under the total order --------------------- */

typedef struct {
  float s32;
  int32_t a, c;
  double s64;
} pred_t;

/* x ranks before y: FP32 score descending, then a, then c ascending */
static inline int better(const pred_t *x, const pred_t *y) {
  if (x->s32 != y->s32) return x->s32 > y->s32;
  if (x->a != y->a) return x->a < y->a;
  return x->c < y->c;
}

static int cmp_pred_desc(const void *x, const void *y) {
  const pred_t *a = (const pred_t *)x, *b = (const pred_t *)y;
  if (better(a, b)) return -1;
  if (better(b, a)) return 1;
  return 0;
}

/* The k best entries offered so far: a buffer of up to 2k entries that is
 * sorted and cut to its first k whenever it fills.  After a cut, the k-th
 * entry is a floor: an entry not better than it cannot be among the final k,
 * so it is not kept. */
typedef struct {
  pred_t *v;
  int64_t n, k;
  int has_floor;
  pred_t floor;
} best_t;

static void best_cut(best_t *b) {
  qsort(b->v, (size_t)b->n, sizeof(pred_t), cmp_pred_desc);
  if (b->n > b->k) b->n = b->k;
  if (b->k > 0 && b->n == b->k) {
    b->floor = b->v[b->k - 1];
    b->has_floor = 1;
  }
}

static void best_offer(best_t *b, pred_t x) {
  if (b->k == 0) return;
  if (b->has_floor && !better(&x, &b->floor)) return;
  if (b->n == 2 * b->k) {
    best_cut(b);
    if (!better(&x, &b->floor)) return;
  }
  b->v[b->n++] = x;
}

static int best_init(best_t *b, int64_t k) {
  b->k = k > 0 ? k : 0;
  b->n = 0;
  b->has_floor = 0;
  b->v = (pred_t *)malloc((size_t)(2 * b->k > 0 ? 2 * b->k : 1) * sizeof(pred_t));
  return b->v != NULL;
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
 * NULL): the candidates owned by those sources, top k of them.  Sources are
 * shared among threads; each thread keeps the k best of its own, and the
 * final list is the k best of the threads' sorted lists, merged. */
int64_t oracle_predict_sources(int64_t n, const int64_t *off, const int32_t *idx, int64_t L,
                               int m, int64_t k, float s_th, int nthreads, const int32_t *sources,
                               int64_t ns, int32_t *out_a, int32_t *out_c, float *out_s32,
                               double *out_s64) {
  int T = get_threads(nthreads);
  best_t *B = (best_t *)calloc((size_t)T, sizeof(best_t));
  int failed = B == NULL;
  for (int t = 0; !failed && t < T; t++)
    if (!best_init(&B[t], k)) failed = 1;
  if (!failed) {
#pragma omp parallel num_threads(T)
    {
#ifdef _OPENMP
      int tid = omp_get_thread_num();
#else
      int tid = 0;
#endif
      sums_t sm;
      if (!sums_init(&sm, n)) {
#pragma omp atomic write
        failed = 1;
      } else {
#pragma omp for schedule(dynamic, 2048)
        for (int64_t i = 0; i < ns; i++) {
          const int64_t a = sources ? sources[i] : i;
          sums_of(&sm, off, idx, L, m, a, 0);
          for (int64_t j = 0; j < sm.ntouched; j++) {
            const int64_t c = sm.touched[j];
            if (!is_candidate(&sm, c)) continue;
            const double s = oracle_score(m, sm.h[c], sm.w[c], deg_of(off, a), deg_of(off, c));
            const float s32 = (float)s;
            if (!(s32 > s_th)) continue; /* strictly above the score threshold */
            pred_t x = {s32, (int32_t)a, (int32_t)c, s};
            best_offer(&B[tid], x);
          }
          sums_clear(&sm, off, idx, a);
        }
      }
      sums_free(&sm);
    }
  }
  int64_t r = 0;
  if (!failed) {
#pragma omp parallel for num_threads(T) schedule(dynamic, 1)
    for (int t = 0; t < T; t++) best_cut(&B[t]);
    /* merge the sorted per-thread lists: repeatedly take the best head */
    int64_t *head = (int64_t *)calloc((size_t)T, sizeof(int64_t));
    while (head && r < k) {
      int pick = -1;
      for (int t = 0; t < T; t++) {
        if (head[t] >= B[t].n) continue;
        if (pick < 0 || better(&B[t].v[head[t]], &B[pick].v[head[pick]])) pick = t;
      }
      if (pick < 0) break;
      const pred_t x = B[pick].v[head[pick]++];
      out_a[r] = x.a;
      out_c[r] = x.c;
      out_s32[r] = x.s32;
      out_s64[r] = x.s64;
      r++;
    }
    if (!head) failed = 1;
    free(head);
  }
  for (int t = 0; B && t < T; t++) free(B[t].v);
  free(B);
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
    sums_t sm;
    best_t bs;
    const int ok_b = best_init(&bs, kq);
    if (!sums_init(&sm, n) || !ok_b) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < ns; i++) {
        const int64_t s = src[i];
        bs.n = 0;
        bs.has_floor = 0;
        sums_of(&sm, off, idx, L, m, s, 1);
        for (int64_t j = 0; j < sm.ntouched; j++) {
          const int64_t c = sm.touched[j];
          if (!is_candidate(&sm, c)) continue;
          const double sc = oracle_score(m, sm.h[c], sm.w[c], deg_of(off, s), deg_of(off, c));
          const float s32 = (float)sc;
          if (!(s32 > s_th)) continue;
          pred_t x = {s32, 0, (int32_t)c, sc}; /* a is the same for all: ties go by c */
          best_offer(&bs, x);
        }
        sums_clear(&sm, off, idx, s);
        best_cut(&bs);
        for (int64_t j = 0; j < bs.n; j++) {
          out_c[i * kq + j] = bs.v[j].c;
          out_s32[i * kq + j] = bs.v[j].s32;
          out_s64[i * kq + j] = bs.v[j].s64;
        }
        out_cnt[i] = (int32_t)bs.n;
      }
    }
    sums_free(&sm);
    if (ok_b) free(bs.v);
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
    sums_t t;
    if (!sums_init(&t, n)) {
#pragma omp atomic write
      failed = 1;
    } else {
#pragma omp for schedule(dynamic, 2048)
      for (int64_t a = 0; a < n; a++) {
        sums_of(&t, off, idx, L, M_CN, a, 0);
        for (int64_t i = 0; i < t.ntouched; i++) {
          const int64_t c = t.touched[i];
          if (!is_candidate(&t, c)) continue;
          cnt += 1;
          sh += (uint64_t)t.h[c];
          sm += fp_mix((uint64_t)a, (uint64_t)c, (uint64_t)t.h[c]);
        }
        for (int64_t e = off[a]; e < off[a + 1]; e++) {
          int64_t b = idx[e];
          if (!explored(off, b, L)) continue;
          for (int64_t f = off[b]; f < off[b + 1]; f++) wed += (idx[f] > a);
        }
        sums_clear(&t, off, idx, a);
      }
    }
    sums_free(&t);
  }
  out[0] = cnt;
  out[1] = sh;
  out[2] = sm;
  out[3] = wed;
  return failed ? -1 : 0;
}

/*
 * synth.c - seeded synthetic graph generators and the observed/unobserved
 * edge split used as inputs by both the CPU oracle and the GPU path.
 *
 * This module holds none of the link-prediction arithmetic: it only makes
 * simple undirected graphs in CSR form (rows sorted ascending, symmetric, no
 * self-loops, no duplicate edges) and splits their edges.
 *
 * Random numbers: a counter-based SplitMix64 stream.  SplitMix64 (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014)
 * outputs mix(s + (i+1)*GOLDEN) for state s and index i, where mix is its
 * 64-bit finaliser.  Stream j of seed s uses the state mix(s + (j+1)*GOLDEN2),
 * so every draw is a pure function of (seed, stream, index) and the result is
 * independent of the number of threads.
 *
 * Generators
 *  - Chung-Lu, edge-sampling form: weights w_i = (i+1)^(-1/(gamma-1)) scaled
 *    to mean avg_deg, optionally capped at w_max (excess redistributed by
 *    rescaling the uncapped weights until stable); m = round(n*avg_deg/2)
 *    endpoint pairs drawn independently with probability proportional to w by
 *    inverse CDF; self-loops and duplicates dropped; vertex ids then permuted
 *    by a seeded Fisher-Yates shuffle.
 *  - R-MAT: 2^scale vertices, edge_factor*2^scale samples, one quadrant choice
 *    per level with probabilities (a, b, c, d), no per-level noise; symmetrised,
 *    self-loops and duplicates dropped, ids permuted as above.
 *  - Holdout: a uniform sample without replacement of round(frac*m) undirected
 *    edges (partial Fisher-Yates over the canonical (u<v, sorted) edge list);
 *    the observed graph is the rest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define GOLDEN2 0xD1B54A32D192ED03ULL

static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t stream_state(uint64_t seed, uint64_t stream) {
  return sm_mix(seed + (stream + 1) * GOLDEN2);
}
static inline uint64_t draw_u64(uint64_t state, uint64_t i) {
  return sm_mix(state + (i + 1) * GOLDEN);
}
/* uniform in [0, 1) with 53 random bits */
static inline double draw_unit(uint64_t state, uint64_t i) {
  return (double)(draw_u64(state, i) >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct {
  int64_t n;
  int64_t nnz; /* arcs = 2 * undirected edges */
  int64_t *off;
  int32_t *idx;
} synth_csr;

void synth_free(synth_csr *g) {
  if (!g) return;
  free(g->off);
  free(g->idx);
  free(g);
}
int64_t synth_n(const synth_csr *g) { return g->n; }
int64_t synth_nnz(const synth_csr *g) { return g->nnz; }
const int64_t *synth_offsets(const synth_csr *g) { return g->off; }
const int32_t *synth_indices(const synth_csr *g) { return g->idx; }

static int cmp_i32(const void *x, const void *y) {
  int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

static void sort_row(int32_t *p, int64_t len) {
  if (len < 32) {
    for (int64_t i = 1; i < len; i++) {
      int32_t v = p[i];
      int64_t j = i - 1;
      while (j >= 0 && p[j] > v) { p[j + 1] = p[j]; j--; }
      p[j + 1] = v;
    }
  } else {
    qsort(p, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

/*
 * Build a simple symmetric CSR from m endpoint pairs (u[i], v[i]); pairs with
 * u == v are dropped, duplicates are removed.  Takes ownership of nothing.
 */
static synth_csr *csr_from_pairs(int64_t n, int64_t m, const int32_t *u, const int32_t *v) {
  int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg) return NULL;
  for (int64_t i = 0; i < m; i++) {
    if (u[i] == v[i]) continue;
    deg[u[i]]++;
    deg[v[i]]++;
  }
  int64_t *start = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  start[0] = 0;
  for (int64_t i = 0; i < n; i++) start[i + 1] = start[i] + deg[i];
  int64_t total = start[n];
  int32_t *tmp = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  int64_t *fill = deg; /* reuse as cursor */
  for (int64_t i = 0; i < n; i++) fill[i] = start[i];
  for (int64_t i = 0; i < m; i++) {
    if (u[i] == v[i]) continue;
    tmp[fill[u[i]]++] = v[i];
    tmp[fill[v[i]]++] = u[i];
  }
  /* sort + dedup every row, count survivors */
  int64_t *keep = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n; r++) {
    int32_t *p = tmp + start[r];
    int64_t len = start[r + 1] - start[r];
    sort_row(p, len);
    int64_t w = 0;
    for (int64_t i = 0; i < len; i++)
      if (w == 0 || p[w - 1] != p[i]) p[w++] = p[i];
    keep[r] = w;
  }
  synth_csr *g = (synth_csr *)malloc(sizeof(synth_csr));
  g->n = n;
  g->off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  g->off[0] = 0;
  for (int64_t r = 0; r < n; r++) g->off[r + 1] = g->off[r] + keep[r];
  g->nnz = g->off[n];
  g->idx = (int32_t *)malloc((size_t)(g->nnz > 0 ? g->nnz : 1) * sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n; r++)
    memcpy(g->idx + g->off[r], tmp + start[r], (size_t)keep[r] * sizeof(int32_t));
  free(deg);
  free(start);
  free(tmp);
  free(keep);
  return g;
}

/* seeded Fisher-Yates permutation of 0..n-1 (stream 'stream' of 'seed') */
static int32_t *random_perm(int64_t n, uint64_t seed, uint64_t stream) {
  int32_t *p = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int64_t i = 0; i < n; i++) p[i] = (int32_t)i;
  uint64_t st = stream_state(seed, stream);
  for (int64_t i = n - 1; i > 0; i--) {
    uint64_t j = draw_u64(st, (uint64_t)i) % (uint64_t)(i + 1);
    int32_t t = p[i];
    p[i] = p[j];
    p[j] = t;
  }
  return p;
}

static void relabel_pairs(int64_t m, int32_t *u, int32_t *v, const int32_t *perm) {
#pragma omp parallel for
  for (int64_t i = 0; i < m; i++) {
    u[i] = perm[u[i]];
    v[i] = perm[v[i]];
  }
}

/* index of the first cumulative weight > x (inverse CDF) */
static inline int64_t upper_bound_d(const double *cum, int64_t n, double x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (cum[mid] > x) hi = mid; else lo = mid + 1;
  }
  return lo < n ? lo : n - 1;
}

synth_csr *synth_chung_lu(int64_t n, double avg_deg, double gamma, double w_max,
                          int64_t n_samples, uint64_t seed) {
  if (n <= 0 || avg_deg <= 0 || gamma <= 1.0) return NULL;
  double *w = (double *)malloc((size_t)n * sizeof(double));
  double ex = -1.0 / (gamma - 1.0), s = 0;
  for (int64_t i = 0; i < n; i++) { w[i] = pow((double)(i + 1), ex); s += w[i]; }
  double target = avg_deg * (double)n;
  for (int64_t i = 0; i < n; i++) w[i] *= target / s;
  if (w_max > 0) {
    /* cap and rescale the uncapped weights until the total is restored */
    for (int it = 0; it < 100; it++) {
      double capped = 0, free_sum = 0;
      int64_t nc = 0;
      for (int64_t i = 0; i < n; i++) {
        if (w[i] >= w_max) { w[i] = w_max; capped += w_max; nc++; } else free_sum += w[i];
      }
      if (nc == 0 || free_sum <= 0) break;
      double f = (target - capped) / free_sum;
      if (fabs(f - 1.0) < 1e-12) break;
      for (int64_t i = 0; i < n; i++) if (w[i] < w_max) w[i] *= f;
    }
  }
  double *cum = (double *)malloc((size_t)n * sizeof(double));
  double acc = 0;
  for (int64_t i = 0; i < n; i++) { acc += w[i]; cum[i] = acc; }
  free(w);
  int64_t m = n_samples > 0 ? n_samples : (int64_t)llround((double)n * avg_deg / 2.0);
  int32_t *u = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  int32_t *v = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  uint64_t st = stream_state(seed, 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; i++) {
    u[i] = (int32_t)upper_bound_d(cum, n, draw_unit(st, 2 * (uint64_t)i) * acc);
    v[i] = (int32_t)upper_bound_d(cum, n, draw_unit(st, 2 * (uint64_t)i + 1) * acc);
  }
  free(cum);
  int32_t *perm = random_perm(n, seed, 2);
  relabel_pairs(m, u, v, perm);
  free(perm);
  synth_csr *g = csr_from_pairs(n, m, u, v);
  free(u);
  free(v);
  return g;
}

synth_csr *synth_rmat(int scale, double edge_factor, double a, double b, double c,
                      uint64_t seed) {
  if (scale <= 0 || scale > 30 || edge_factor <= 0) return NULL;
  int64_t n = (int64_t)1 << scale;
  int64_t m = (int64_t)llround(edge_factor * (double)n);
  double ab = a + b, abc = a + b + c;
  int32_t *u = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  int32_t *v = (int32_t *)malloc((size_t)m * sizeof(int32_t));
  uint64_t st = stream_state(seed, 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; i++) {
    int64_t r = 0, col = 0;
    for (int l = 0; l < scale; l++) {
      double x = draw_unit(st, (uint64_t)i * (uint64_t)scale + (uint64_t)l);
      int rb = 0, cb = 0;
      if (x < a) { rb = 0; cb = 0; }
      else if (x < ab) { rb = 0; cb = 1; }
      else if (x < abc) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      r = (r << 1) | rb;
      col = (col << 1) | cb;
    }
    u[i] = (int32_t)r;
    v[i] = (int32_t)col;
  }
  int32_t *perm = random_perm(n, seed, 2);
  relabel_pairs(m, u, v, perm);
  free(perm);
  synth_csr *g = csr_from_pairs(n, m, u, v);
  free(u);
  free(v);
  return g;
}

/* CSR from an explicit undirected edge list (u[i], v[i]); loops/dups dropped */
synth_csr *synth_from_edges(int64_t n, int64_t m, const int32_t *u, const int32_t *v) {
  for (int64_t i = 0; i < m; i++)
    if (u[i] < 0 || v[i] < 0 || u[i] >= n || v[i] >= n) return NULL;
  return csr_from_pairs(n, m, u, v);
}

/*
 * Remove round(frac * m) uniformly chosen undirected edges.  Writes the removed
 * edges (u < v) to held_u/held_v (capacity *n_held, which returns the count)
 * and returns the observed graph.
 */
synth_csr *synth_holdout(const synth_csr *g, double frac, uint64_t seed,
                         int32_t *held_u, int32_t *held_v, int64_t *n_held) {
  int64_t m = g->nnz / 2;
  int32_t *eu = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t *ev = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int64_t t = 0;
  for (int64_t r = 0; r < g->n; r++)
    for (int64_t e = g->off[r]; e < g->off[r + 1]; e++)
      if (g->idx[e] > r) { eu[t] = (int32_t)r; ev[t] = g->idx[e]; t++; }
  int64_t k = (int64_t)llround(frac * (double)m);
  if (k > m) k = m;
  if (k > *n_held) { free(eu); free(ev); return NULL; }
  uint64_t st = stream_state(seed, 3);
  /* partial Fisher-Yates: the first k slots become the sample */
  for (int64_t i = 0; i < k; i++) {
    uint64_t j = (uint64_t)i + draw_u64(st, (uint64_t)i) % (uint64_t)(m - i);
    int32_t x = eu[i]; eu[i] = eu[j]; eu[j] = x;
    x = ev[i]; ev[i] = ev[j]; ev[j] = x;
  }
  memcpy(held_u, eu, (size_t)k * sizeof(int32_t));
  memcpy(held_v, ev, (size_t)k * sizeof(int32_t));
  *n_held = k;
  synth_csr *o = csr_from_pairs(g->n, m - k, eu + k, ev + k);
  free(eu);
  free(ev);
  return o;
}

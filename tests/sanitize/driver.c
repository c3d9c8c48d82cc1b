/*
 * Host-only driver for a sanitizer build (AddressSanitizer and
 * UndefinedBehaviorSanitizer, gcc) of the CPU oracle and the input
 * generators: it makes small seeded graphs and runs every oracle entry point
 * on them, so that an out-of-bounds access, a use of freed memory or an
 * undefined operation in either file stops the run.  Built and run by
 * tests/test_sanitize.py; nothing here is part of the library.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct synth_csr synth_csr;
synth_csr *synth_chung_lu(int64_t n, double avg_deg, double gamma, double w_max, int64_t m_target,
                          uint64_t seed);
synth_csr *synth_rmat(int scale, double edge_factor, double a, double b, double c, uint64_t seed);
synth_csr *synth_from_edges(int64_t n, int64_t m, const int32_t *u, const int32_t *v);
synth_csr *synth_holdout(const synth_csr *g, double frac, uint64_t seed, int32_t *held_u, int32_t *held_v,
                         int64_t *n_held);
void synth_free(synth_csr *g);
int64_t synth_n(const synth_csr *g);
int64_t synth_nnz(const synth_csr *g);
const int64_t *synth_offsets(const synth_csr *g);
const int32_t *synth_indices(const synth_csr *g);

double oracle_weight(int m, int64_t db);
double oracle_score(int m, int64_t h, double w, int64_t da, int64_t dc);
int oracle_pair(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m, int64_t a, int64_t c,
                int64_t *h_out, double *s_out);
void oracle_pairs(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m, const int32_t *a,
                  const int32_t *c, int64_t np, int nthreads, int8_t *ok, int64_t *h_out, double *s_out);
int64_t oracle_bruteforce(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m, int32_t *out_a,
                          int32_t *out_c, int64_t *out_h, double *out_s, int64_t cap);
int64_t oracle_source(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m, int64_t a, int mode,
                      int32_t *out_c, int64_t *out_h, double *out_s, int64_t cap);
int64_t oracle_predict(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m, int64_t k,
                       float s_th, int nthreads, int32_t *out_a, int32_t *out_c, float *out_s32,
                       double *out_s64);
int64_t oracle_predict_sources(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m, int64_t k,
                               float s_th, int nthreads, const int32_t *sources, int64_t ns, int32_t *out_a,
                               int32_t *out_c, float *out_s32, double *out_s64);
int oracle_query(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int m, const int32_t *src,
                 int64_t ns, int32_t kq, float s_th, int nthreads, int32_t *out_c, float *out_s32,
                 double *out_s64, int32_t *out_cnt);
int oracle_fingerprint(int64_t n, const int64_t *off, const int32_t *idx, int64_t L, int nthreads, uint64_t *out);

#define CHECK(x)                                                   \
  do {                                                             \
    if (!(x)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static int exercise(const synth_csr *g) {
  const int64_t n = synth_n(g);
  const int64_t *off = synth_offsets(g);
  const int32_t *idx = synth_indices(g);
  const int64_t limits[3] = {2, 16, INT64_MAX};
  int64_t k = 50;
  int32_t *a = malloc(sizeof(int32_t) * (size_t)(n * n + 1)), *c = malloc(sizeof(int32_t) * (size_t)(n * n + 1));
  int64_t *h = malloc(sizeof(int64_t) * (size_t)(n * n + 1));
  double *s = malloc(sizeof(double) * (size_t)(n * n + 1));
  float *s32 = malloc(sizeof(float) * (size_t)(n * n + 1));
  int8_t *ok = malloc((size_t)(n * n + 1));
  int32_t *cnt = malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *src = malloc(sizeof(int32_t) * (size_t)(n + 1));
  CHECK(a && c && h && s && s32 && ok && cnt && src);
  for (int64_t i = 0; i < n; i++) src[i] = (int32_t)i;
  for (int li = 0; li < 3; li++) {
    for (int m = 0; m < 9; m++) {
      const int64_t L = limits[li];
      const int64_t tot = oracle_bruteforce(n, off, idx, L, m, a, c, h, s, n * n);
      CHECK(tot >= 0 && tot <= n * n);
      {  // a capacity below the total, in buffers of exactly that size
        const int64_t cap = tot / 2;
        int32_t *a2 = malloc(sizeof(int32_t) * (size_t)cap), *c2 = malloc(sizeof(int32_t) * (size_t)cap);
        int64_t *h2 = malloc(sizeof(int64_t) * (size_t)cap);
        double *s2 = malloc(sizeof(double) * (size_t)cap);
        CHECK(cap == 0 || (a2 && c2 && h2 && s2));
        CHECK(oracle_bruteforce(n, off, idx, L, m, a2, c2, h2, s2, cap) == tot);
        free(a2); free(c2); free(h2); free(s2);
      }
      oracle_pairs(n, off, idx, L, m, a, c, tot, 2, ok, h, s);
      for (int64_t i = 0; i < tot; i++) CHECK(ok[i]);
      const int64_t r = oracle_predict(n, off, idx, L, m, k, 0.0f, 3, a, c, s32, s);
      CHECK(r >= 0 && r <= k);
      const int64_t rs = oracle_predict_sources(n, off, idx, L, m, k, 0.0f, 2, src, n / 2, a, c, s32, s);
      CHECK(rs >= 0 && rs <= k);
      CHECK(oracle_query(n, off, idx, L, m, src, n, 4, 0.0f, 2, c, s32, s, cnt) == 0);
      for (int64_t v = 0; v < n; v += 7) {
        const int64_t q = oracle_source(n, off, idx, L, m, v, v & 1, c, h, s, n);
        CHECK(q >= 0 && q <= n);
      }
    }
    uint64_t fp[4];
    CHECK(oracle_fingerprint(n, off, idx, limits[li], 2, fp) == 0);
  }
  free(a); free(c); free(h); free(s); free(s32); free(ok); free(cnt); free(src);
  return 0;
}

int main(void) {
  synth_csr *cl = synth_chung_lu(300, 8.0, 2.2, 0.0, 0, 7);
  CHECK(cl != NULL);
  int32_t hu[4096], hv[4096];
  int64_t nh = 4096;  /* capacity of hu / hv on entry, count on return */
  synth_csr *obs = synth_holdout(cl, 0.1, 7, hu, hv, &nh);
  CHECK(obs != NULL && nh > 0);
  synth_csr *rm = synth_rmat(8, 8.0, 0.57, 0.19, 0.19, 3);
  CHECK(rm != NULL);
  const int32_t eu[5] = {0, 0, 1, 2, 3}, ev[5] = {1, 2, 2, 3, 4};
  synth_csr *small = synth_from_edges(6, 5, eu, ev);  // vertex 5 isolated
  CHECK(small != NULL);
  synth_csr *empty = synth_from_edges(0, 0, eu, ev);
  CHECK(empty != NULL);
  if (exercise(obs) || exercise(rm) || exercise(small) || exercise(empty)) return 1;
  synth_free(cl); synth_free(obs); synth_free(rm); synth_free(small); synth_free(empty);
  puts("sanitized run ok");
  return 0;
}

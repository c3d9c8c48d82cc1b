// api.hip - the C ABI (include/lp.h): argument checking, device selection,
// the per-graph busy flag, and dispatch to the device code.
#include <cmath>
#include <new>

#include "lp_common.h"

namespace lp {
lp_status build_graph(int64_t n, const int64_t* offsets, const int32_t* indices, uint32_t flags,
                      lp_graph* g);
void destroy_graph(lp_graph* g);
lp_status run_predict(lp_graph* g, int m, int64_t L, int64_t k, float s_th, int32_t* out_a,
                      int32_t* out_c, float* out_score, int64_t* out_count, hipStream_t st);
lp_status run_fingerprint(lp_graph* g, int64_t L, uint64_t* out, hipStream_t st);
lp_status run_predict_multi(lp_graph* g, int64_t ng, const int64_t* vstart, const int64_t* kk, int m,
                            int64_t L, float s_th, int32_t* out_a, int32_t* out_c, float* out_score,
                            int64_t* out_count, hipStream_t st);
lp_status run_query(lp_graph* g, Workspace& w, const int32_t* sources, int64_t nq, int m, int64_t L,
                    int32_t kq,
                    float s_th, int32_t* out_c, float* out_score, int32_t* out_count,
                    hipStream_t st);
const char* last_error_text();
}  // namespace lp

using namespace lp;

namespace {

struct BusyGuard {
  lp_graph* g;
  bool ok;
  explicit BusyGuard(lp_graph* gg) : g(gg) {
    int expected = 0;
    ok = g->busy.compare_exchange_strong(expected, 1);
  }
  ~BusyGuard() {
    if (ok) g->busy.store(0);
  }
};

lp_status select_device(const lp_graph* g) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(LP_ERR_DEVICE, "no HIP device");
  }
  if (cur != g->device) LP_HIP(hipSetDevice(g->device));
  return LP_OK;
}

lp_status check_common(lp_graph* g, int m, int64_t L, float s_th) {
  if (!g) return set_error(LP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (m < LP_CN || m > LP_RA) return set_error(LP_ERR_INVALID_ARGUMENT, "measure %d out of range", m);
  if (L < 0) return set_error(LP_ERR_INVALID_ARGUMENT, "hub_limit must be >= 0");
  if (!std::isfinite(s_th) || s_th < 0.0f)
    return set_error(LP_ERR_INVALID_ARGUMENT, "score_threshold must be finite and >= 0");
  return LP_OK;
}

template <class F>
lp_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return set_error(LP_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return set_error(LP_ERR_DEVICE, "unexpected exception");
  }
}

}  // namespace

extern "C" {

lp_status lp_graph_create(int64_t n, const int64_t* offsets, const int32_t* indices, uint32_t flags,
                          lp_graph** out) {
  clear_error();
  return guarded([&]() -> lp_status {
    if (!out) return set_error(LP_ERR_INVALID_ARGUMENT, "out is NULL");
    if (n < 0 || n > INT32_MAX) return set_error(LP_ERR_INVALID_ARGUMENT, "n must be in [0, 2^31 - 1]");
    if (!offsets) return set_error(LP_ERR_INVALID_ARGUMENT, "offsets is NULL");
    if (flags & ~(uint32_t)LP_VALIDATE) return set_error(LP_ERR_INVALID_ARGUMENT, "unknown flags");
    lp_graph* g = new lp_graph();
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      delete g;
      return set_error(LP_ERR_DEVICE, "no HIP device");
    }
    g->device = dev;
    lp_status s = build_graph(n, offsets, indices, flags, g);
    if (s != LP_OK) {
      destroy_graph(g);
      delete g;
      return s;
    }
    *out = g;
    return LP_OK;
  });
}

lp_status lp_graph_destroy(lp_graph* g) {
  clear_error();
  if (!g) return LP_OK;
  (void)select_device(g);
  (void)hipDeviceSynchronize();
  destroy_graph(g);
  delete g;
  return LP_OK;
}

lp_status lp_graph_info(const lp_graph* g, int64_t* n, int64_t* arcs, int64_t* max_degree,
                        int64_t* device_bytes) {
  clear_error();
  if (!g) return set_error(LP_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (n) *n = g->n;
  if (arcs) *arcs = g->arcs;
  if (max_degree) *max_degree = g->max_deg;
  if (device_bytes) *device_bytes = g->device_bytes;
  return LP_OK;
}

lp_status lp_predict(lp_graph* g, lp_measure m, int64_t hub_limit, int64_t k, float score_threshold,
                     int32_t* out_a, int32_t* out_c, float* out_score, int64_t* out_count,
                     void* hip_stream) {
  clear_error();
  if (out_count) *out_count = 0;
  return guarded([&]() -> lp_status {
    LP_TRY(check_common(g, (int)m, hub_limit, score_threshold));
    if (!out_count) return set_error(LP_ERR_INVALID_ARGUMENT, "out_count is NULL");
    if (k < 0) return set_error(LP_ERR_INVALID_ARGUMENT, "k must be >= 0");
    if (k > 0 && (!out_a || !out_c || !out_score))
      return set_error(LP_ERR_INVALID_ARGUMENT, "output pointer is NULL");
    BusyGuard busy(g);
    if (!busy.ok) return set_error(LP_ERR_BUSY, "graph is in use by another thread");
    LP_TRY(select_device(g));
    ScratchLimit limit(g->tuning.scratch_limit);
    return run_predict(g, (int)m, hub_limit, k, score_threshold, out_a, out_c, out_score, out_count,
                       (hipStream_t)hip_stream);
  });
}

lp_status lp_predict_multi(lp_graph* g, int64_t ngraphs, const int64_t* vstart, const int64_t* k,
                           lp_measure m, int64_t hub_limit, float score_threshold, int32_t* out_a,
                           int32_t* out_c, float* out_score, int64_t* out_count, void* hip_stream) {
  clear_error();
  return guarded([&]() -> lp_status {
    LP_TRY(check_common(g, (int)m, hub_limit, score_threshold));
    if (ngraphs < 1 || ngraphs > INT32_MAX)
      return set_error(LP_ERR_INVALID_ARGUMENT, "ngraphs must be in [1, 2^31 - 1]");
    if (!vstart || !k || !out_count) return set_error(LP_ERR_INVALID_ARGUMENT, "array pointer is NULL");
    if (vstart[0] != 0 || vstart[ngraphs] != g->n)
      return set_error(LP_ERR_INVALID_ARGUMENT, "vstart must run from 0 to n");
    uint64_t ktot = 0;
    for (int64_t i = 0; i < ngraphs; i++) {
      if (vstart[i + 1] < vstart[i]) return set_error(LP_ERR_INVALID_ARGUMENT, "vstart decreases");
      if (k[i] < 0) return set_error(LP_ERR_INVALID_ARGUMENT, "k[%lld] < 0", (long long)i);
      ktot += (uint64_t)k[i];
    }
    if (ktot >= (1ull << 32)) return set_error(LP_ERR_INVALID_ARGUMENT, "sum of k too large");
    if (ktot > 0 && (!out_a || !out_c || !out_score))
      return set_error(LP_ERR_INVALID_ARGUMENT, "output pointer is NULL");
    BusyGuard busy(g);
    if (!busy.ok) return set_error(LP_ERR_BUSY, "graph is in use by another thread");
    LP_TRY(select_device(g));
    ScratchLimit limit(g->tuning.scratch_limit);
    return run_predict_multi(g, ngraphs, vstart, k, (int)m, hub_limit, score_threshold, out_a, out_c,
                             out_score, out_count, (hipStream_t)hip_stream);
  });
}

lp_status lp_query(lp_graph* g, const int32_t* sources, int64_t n_sources, lp_measure m,
                   int64_t hub_limit, int32_t k_q, float score_threshold, int32_t* out_c,
                   float* out_score, int32_t* out_count, void* hip_stream) {
  clear_error();
  return guarded([&]() -> lp_status {
    LP_TRY(check_common(g, (int)m, hub_limit, score_threshold));
    if (n_sources < 0 || n_sources > INT32_MAX)
      return set_error(LP_ERR_INVALID_ARGUMENT, "n_sources must be in [0, 2^31 - 1]");
    if (k_q <= 0) return set_error(LP_ERR_INVALID_ARGUMENT, "k_q must be > 0");
    if ((uint64_t)n_sources * (uint64_t)k_q >= (1ull << 32))
      return set_error(LP_ERR_INVALID_ARGUMENT, "n_sources * k_q too large");
    if (n_sources > 0 && (!sources || !out_c || !out_score || !out_count))
      return set_error(LP_ERR_INVALID_ARGUMENT, "array pointer is NULL");
    BusyGuard busy(g);
    if (!busy.ok) return set_error(LP_ERR_BUSY, "graph is in use by another thread");
    LP_TRY(select_device(g));
    ScratchLimit limit(g->tuning.scratch_limit);
    return run_query(g, g->ws, sources, n_sources, (int)m, hub_limit, k_q, score_threshold, out_c,
                     out_score, out_count, (hipStream_t)hip_stream);
  });
}

lp_status lp_fingerprint(lp_graph* g, int64_t hub_limit, uint64_t* out, void* hip_stream) {
  clear_error();
  return guarded([&]() -> lp_status {
    LP_TRY(check_common(g, LP_CN, hub_limit, 0.0f));
    if (!out) return set_error(LP_ERR_INVALID_ARGUMENT, "out is NULL");
    BusyGuard busy(g);
    if (!busy.ok) return set_error(LP_ERR_BUSY, "graph is in use by another thread");
    LP_TRY(select_device(g));
    ScratchLimit limit(g->tuning.scratch_limit);
    return run_fingerprint(g, hub_limit, out, (hipStream_t)hip_stream);
  });
}

lp_status lp_set_tuning(lp_graph* g, const lp_tuning* t) {
  clear_error();
  if (!g || !t) return set_error(LP_ERR_INVALID_ARGUMENT, "NULL argument");
  if (t->lds_wedge_cap < 0 || t->global_slots < 0 || t->scratch_limit < 0)
    return set_error(LP_ERR_INVALID_ARGUMENT, "tuning values must be >= 0");
  for (int b = 0; b < 5; b++)
    if (t->bucket_max[b] < 0 || t->bucket_max[b] > lp::kBucketMaxDefault[b])
      return set_error(LP_ERR_INVALID_ARGUMENT, "bucket_max[b] must lie in [0, its default]");
  if ((t->batch_sources[0] != 0 && t->batch_sources[0] != 48 && t->batch_sources[0] != 32) ||
      (t->batch_sources[1] != 0 && t->batch_sources[1] != 8 && t->batch_sources[1] != 4))
    return set_error(LP_ERR_INVALID_ARGUMENT, "batch_sources: tiny 48 or 32, small 8 or 4");
  if (t->kernel_shape[0] < 0 || t->kernel_shape[0] > 4 || t->kernel_shape[1] < 0 || t->kernel_shape[1] > 4 ||
      t->kernel_shape[1] == 2)
    return set_error(LP_ERR_INVALID_ARGUMENT, "kernel_shape: small 0-4, mid1 0, 1, 3 or 4");
  g->tuning = *t;
  return LP_OK;
}

lp_status lp_last_stats(const lp_graph* g, lp_stats* out) {
  clear_error();
  if (!g || !out) return set_error(LP_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = g->last;
  return LP_OK;
}

const char* lp_status_string(lp_status s) {
  switch (s) {
    case LP_OK: return "LP_OK";
    case LP_ERR_INVALID_ARGUMENT: return "LP_ERR_INVALID_ARGUMENT";
    case LP_ERR_INVALID_GRAPH: return "LP_ERR_INVALID_GRAPH";
    case LP_ERR_OUT_OF_MEMORY: return "LP_ERR_OUT_OF_MEMORY";
    case LP_ERR_DEVICE: return "LP_ERR_DEVICE";
    case LP_ERR_BUSY: return "LP_ERR_BUSY";
    default: return "LP_ERR_UNKNOWN";
  }
}

const char* lp_last_error(void) { return last_error_text(); }

}  // extern "C"

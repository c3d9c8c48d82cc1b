// static_query.hip - lp_query_static: the per-source query of lp_query with
// every piece of device scratch taken from one fixed array of this library,
// for callers that cannot allocate device memory during a call (tight
// serving loops, hosts that forbid hipMalloc after start-up).  The graph
// itself is created beforehand.
#include <atomic>
#include <mutex>

#include "lp_common.h"

namespace lp {
lp_status run_query(lp_graph* g, Workspace& w, const int32_t* sources, int64_t nq, int m, int64_t L,
                    int32_t kq, float s_th, int32_t* out_c, float* out_score, int32_t* out_count,
                    hipStream_t st);
}  // namespace lp

using namespace lp;

namespace {

// Shares of the scratch array, in bytes (each a multiple of 256).  The limits
// of lp_query_static follow from them: at most kMaxSources sources per call,
// n_sources * k_q <= kMaxRows, a two-hop path bound (the candidate capacity)
// of at most kMaxPaths, and sources above the LDS capacity only on graphs
// whose dense accumulator (12 bytes per vertex) fits kGlobalBytes.
constexpr size_t kMaxSources = 4096;
constexpr size_t kMaxPaths = size_t(1) << 21;
constexpr size_t kMaxRows = size_t(1) << 20;
constexpr size_t kMB = size_t(1) << 20;

constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t max2(size_t a, size_t b) { return a > b ? a : b; }

constexpr size_t kSrcBytes = align256(kMaxSources * 4);
constexpr size_t kRowsBytes = align256(kMaxSources * 64 * 7 + 256);  // source records per bucket
constexpr size_t kStatsBytes = 4096;
constexpr size_t kCountersBytes = align256(4096 + (size_t(1) << 16) * (4 + 64));  // counters, overflow list
constexpr size_t kCandBytes = align256(kMaxPaths * 4);                         // one word per candidate
constexpr size_t kSegBytes = align256(kMaxSources * 8 + 64);
// sort words; the first also stages the outputs for host pointers
constexpr size_t kSortBytes = max2(kCandBytes, align256(kMaxRows * 8 + kMaxSources * 4 + 64));
constexpr size_t kSortCountsBytes = align256((kMaxPaths / 2048 + 1) * 256 * 4 * 2);
constexpr size_t kScanBytes = 256 * 1024;
constexpr size_t kGlobalBytes = 32 * kMB;  // dense accumulator slabs
constexpr size_t kSpaMetaBytes = kMB;      // their per-round metadata
constexpr size_t kScratchBytes = kSrcBytes + kRowsBytes + kStatsBytes + kCountersBytes + 3 * kCandBytes +
                                 kSegBytes + 3 * kSortBytes + kSortCountsBytes + kScanBytes + kGlobalBytes +
                                 kSpaMetaBytes;
static_assert(kScratchBytes <= 96 * kMB, "the fixed scratch stays within 96 MiB");

constexpr int kMaxDevices = 64;

}  // namespace

// The fixed scratch: one copy per device, held until the process ends.  In
// host code this name only stands in for the device array; the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

struct DeviceScratch {
  std::once_flag once;
  lp_status init_status = LP_OK;
  uint8_t* ptr = nullptr;  // device address of `scratch` on this device
  Workspace ws;            // its buffers carved from ptr, never reallocated or freed
  uint8_t host_stage[4096];
  std::atomic<int> busy{0};
};

DeviceScratch g_dev[kMaxDevices];

void carve(DevBuf& b, uint8_t*& at, size_t bytes) {
  b.p = at;
  b.cap = bytes;
  b.fixed = true;
  at += bytes;
}

// With device `dev` current: the scratch's device address, and the workspace
// over it.  Buffers the query path does not use get no memory (a request
// that would need them fails).
lp_status init_device(DeviceScratch& d) {
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return set_error(LP_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  }
  d.ptr = static_cast<uint8_t*>(p);
  Workspace& w = d.ws;
  uint8_t* at = d.ptr;
  carve(w.q_src, at, kSrcBytes);
  carve(w.q_rows, at, kRowsBytes);
  carve(w.stats, at, kStatsBytes);
  carve(w.counters, at, kCountersBytes);
  carve(w.cand_s, at, kCandBytes);
  carve(w.cand_a, at, kCandBytes);
  carve(w.cand_c, at, kCandBytes);
  carve(w.q_cnt, at, kSegBytes);
  for (int i = 0; i < 3; i++) carve(w.sort_tmp[i], at, kSortBytes);
  carve(w.sort_counts, at, kSortCountsBytes);
  carve(w.scan_tmp, at, kScanBytes);
  carve(w.global_tab, at, kGlobalBytes);
  carve(w.spa_meta, at, kSpaMetaBytes);
  if ((size_t)(at - d.ptr) != kScratchBytes) return set_error(LP_ERR_DEVICE, "scratch layout");
  // the remaining buffers of a workspace stay empty and fixed: nothing grows
  DevBuf* none[] = {&w.cnt,      &w.wedges,   &w.lists,     &w.tmp_s[0],   &w.tmp_s[1], &w.tmp_a[0],
                    &w.tmp_a[1], &w.tmp_c[0], &w.tmp_c[1],  &w.hist,       &w.sel_state, &w.sort_tmp[3],
                    &w.unfit,    &w.kept,      &w.q_wedges, &w.q_out,     &w.m_graph,    &w.m_gid,    &w.m_lists};
  for (DevBuf* b : none) {
    b->p = d.ptr;  // non-null so that a zero-byte request succeeds; cap 0 refuses any other
    b->cap = 0;
    b->fixed = true;
  }
  w.host_stats.p = d.host_stage;
  w.host_stats.cap = sizeof(d.host_stage);
  w.host_stats.fixed = true;
  return LP_OK;
}

}  // namespace

extern "C" lp_status lp_query_static(lp_graph* g, const int32_t* sources, int64_t n_sources, lp_measure m,
                                     int64_t hub_limit, int32_t k_q, float score_threshold, int32_t* out_c,
                                     float* out_score, int32_t* out_count, void* hip_stream) {
  clear_error();
  try {
    if (!g) return set_error(LP_ERR_INVALID_ARGUMENT, "graph is NULL");
    if ((int)m < LP_CN || (int)m > LP_RA) return set_error(LP_ERR_INVALID_ARGUMENT, "measure out of range");
    if (hub_limit < 0) return set_error(LP_ERR_INVALID_ARGUMENT, "hub_limit must be >= 0");
    if (!(score_threshold >= 0.0f) || score_threshold > 3.4e38f)
      return set_error(LP_ERR_INVALID_ARGUMENT, "score_threshold must be finite and >= 0");
    if (n_sources < 0 || (uint64_t)n_sources > kMaxSources)
      return set_error(LP_ERR_INVALID_ARGUMENT, "n_sources must be in [0, %zu] (fixed scratch)", kMaxSources);
    if (k_q <= 0) return set_error(LP_ERR_INVALID_ARGUMENT, "k_q must be > 0");
    if ((uint64_t)n_sources * (uint64_t)k_q > kMaxRows)
      return set_error(LP_ERR_INVALID_ARGUMENT, "n_sources * k_q must be <= %zu (fixed scratch)", kMaxRows);
    if (n_sources > 0 && (!sources || !out_c || !out_score || !out_count))
      return set_error(LP_ERR_INVALID_ARGUMENT, "array pointer is NULL");
    if (g->device < 0 || g->device >= kMaxDevices)
      return set_error(LP_ERR_INVALID_ARGUMENT, "device %d beyond the scratch table", g->device);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(LP_ERR_DEVICE, "no HIP device");
    }
    if (cur != g->device && hipSetDevice(g->device) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(LP_ERR_DEVICE, "hipSetDevice(%d) failed", g->device);
    }
    DeviceScratch& d = g_dev[g->device];
    std::call_once(d.once, [&] { d.init_status = init_device(d); });
    if (d.init_status != LP_OK) return set_error(d.init_status, "fixed scratch unavailable on device %d", g->device);
    // one call at a time per device: the scratch is shared by every graph on it
    struct Claim {
      std::atomic<int>& flag;
      bool ok;
      explicit Claim(std::atomic<int>& f) : flag(f) {
        int expected = 0;
        ok = flag.compare_exchange_strong(expected, 1);
      }
      ~Claim() {
        if (ok) flag.store(0);
      }
    } claim(d.busy);
    if (!claim.ok)
      return set_error(LP_ERR_BUSY, "the fixed scratch of device %d is in use by another call", g->device);
    // the slabs of the dense accumulator are cleared again by the first call
    // that needs them: the array keeps whatever the last call (on any graph
    // of this device) left in it
    d.ws.global_slabs = 0;
    const lp_status s = run_query(g, d.ws, sources, n_sources, (int)m, hub_limit, k_q, score_threshold, out_c,
                                  out_score, out_count, (hipStream_t)hip_stream);
    // a call that stopped early may have left work on the stream: it ends
    // before the scratch is released to the next call (which may use
    // another stream)
    if (s != LP_OK && hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) (void)hipGetLastError();
    return s;
  } catch (...) {
    return set_error(LP_ERR_DEVICE, "unexpected exception");
  }
}

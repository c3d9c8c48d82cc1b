// lp_common.h - internal definitions shared by the HIP translation units of
// liblp.so: error handling, device buffers, the resident graph object and the
// entry points of the device primitives.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lp.h"

namespace lp {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------

lp_status set_error(lp_status s, const char* fmt, ...);
lp_status from_hip(hipError_t e, const char* what);
void clear_error();

#define LP_TRY(expr)                          \
  do {                                        \
    lp_status _s = (expr);                    \
    if (_s != LP_OK) return _s;               \
  } while (0)

#define LP_HIP(expr)                                   \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return ::lp::from_hip(_e, #expr); \
  } while (0)

// ---------------------------------------------------------------------------
// Device memory
// ---------------------------------------------------------------------------

// A growable device allocation.  ensure() keeps the contents only when no
// reallocation is needed.  A fixed buffer is a view of memory owned
// elsewhere: ensure() never allocates and fails (LP_ERR_INVALID_ARGUMENT)
// when asked for more than cap; release() leaves it alone.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool fixed = false;
  lp_status ensure(size_t bytes);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Pinned host staging for small device -> host reads (fixed: as for DevBuf).
struct HostBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool fixed = false;
  lp_status ensure(size_t bytes);
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Largest single scratch allocation the calling thread's current call may
// make (0: no limit); a call sets it from its graph's tuning, so that running
// out of device memory can be forced from the host.
struct ScratchLimit {
  static thread_local size_t bytes;
  size_t saved;
  explicit ScratchLimit(int64_t limit) : saved(bytes) { bytes = limit > 0 ? (size_t)limit : 0; }
  ~ScratchLimit() { bytes = saved; }
};

// ---------------------------------------------------------------------------
// Resident graph.  Vertices are relabelled by ascending (degree, original id);
// "new" ids below are ranks in that order.  Ownership of an unordered pair by
// its lower-ranked endpoint leaves every candidate, count and score unchanged
// (a pair is reported with original ids) but makes the large-degree endpoint
// the one that does little work.
// ---------------------------------------------------------------------------

constexpr int kNumBuckets = 7;  // scheduling buckets of the accumulation
constexpr int kStatRows = 8;    // per-launch statistics rows: the buckets, then "split"

struct Workspace {
  // plan
  DevBuf cnt, wedges, lists, counters, stats;
  // candidate buffers (score bits, original a, original c) and selection
  DevBuf cand_s, cand_a, cand_c;
  DevBuf tmp_s[2], tmp_a[2], tmp_c[2];
  DevBuf hist, sel_state, sort_tmp[4], sort_counts, scan_tmp;
  DevBuf global_tab, spa_meta;
  DevBuf unfit;  // packed AA / RA calls: sources whose sums do not fit a packed slot
  DevBuf kept;   // AA / RA with a threshold: batched-bucket sources that can reach it
  unsigned global_slabs = 0;  // accumulator slabs in global_tab
  // query
  DevBuf q_src, q_cnt, q_wedges, q_rows, q_out;
  // several graphs at once: per-graph tables, candidate graph ids, the
  // bucket lists split into sample and rest
  DevBuf m_graph, m_gid, m_lists;
  std::vector<uint32_t> m_checked;  // graph boundaries already checked for joining edges
  HostBuf host_stats;
  // side streams for the concurrent launches of a sampling phase (default
  // priority), forked from and joined back to the caller's stream
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSide] = {};
  // timing events of a call (per-launch clock, phase timer), created once
  hipEvent_t clock_ev[4 * (kNumBuckets + 2)] = {};
  hipEvent_t timer_ev[4] = {};
};

}  // namespace lp

struct lp_graph {
  int device = 0;
  int64_t n = 0;
  int64_t arcs = 0;
  int64_t max_deg = 0;
  int fixed_shift = 40;  // AA/RA sums are accumulated as fixed point with this many fraction bits
  // device arrays in the relabelled id space
  uint32_t* off = nullptr;       // n+1 row offsets
  uint32_t* adj = nullptr;       // arcs, each row ascending
  // two-hop arc list: for every source a, the arcs a->b (b ascending) whose row
  // b holds at least one id > a, i.e. that contribute wedges a-b-c with c > a
  uint32_t* hoff = nullptr;    // n+1 offsets into the list
  uint32_t* hdeg = nullptr;    // degree of b (non-decreasing within a source: ids follow degree)
  uint32_t* hstart = nullptr;  // first position in adj (row b) holding an id > a
  uint32_t* hpsum = nullptr;   // inclusive running total of those suffix lengths within the row
  int64_t harcs = 0;
  uint32_t* deg = nullptr;       // n, non-decreasing
  uint32_t* below = nullptr;     // n, number of neighbours with a smaller id
  uint32_t* deg_first = nullptr; // deg_cap + 1 entries: first new id whose degree is >= d
  uint32_t deg_cap = 0;
  uint32_t* perm = nullptr;      // n, new id -> original id
  uint32_t* rank = nullptr;      // n, original id -> new id
  std::vector<uint32_t> host_deg;  // copy of deg (sorted), for hub boundaries
  int64_t device_bytes = 0;
  lp::Workspace ws;
  lp_tuning tuning{};
  lp_stats last{};
  std::atomic<int> busy{0};
};

namespace lp {

// Number of relabelled vertices whose degree is <= L (they form a prefix).
uint32_t hub_start(const lp_graph* g, int64_t L);

// ---------------------------------------------------------------------------
// Device primitives (prim.hip)
// ---------------------------------------------------------------------------

// scratch bytes that a scan of n entries needs (either scan below)
size_t scan_scratch_bytes(int64_t n);
// exclusive scan of n uint32 into out (n entries), optional total
lp_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, DevBuf& tmp,
                             hipStream_t st);
// inclusive scan of n uint32 into uint64 out
lp_status scan_inclusive_u32_u64(const uint32_t* in, uint64_t* out, int64_t n, DevBuf& tmp,
                                 hipStream_t st);

// Stable LSD radix sort of n records with up to three uint32 words, ordered
// ascending by the (possibly complemented) key words, most significant first.
struct SortSpec {
  uint32_t* w[4];       // record words (sorted in place)
  int nwords;           // 1..4
  int nkeys;            // the first nkeys words are the key, word 0 most significant
  int key_bits[4];      // significant bits per key word (<= 32)
  bool invert[4];       // complement this key word (descending order)
};
lp_status radix_sort(const SortSpec& spec, int64_t n, DevBuf tmp[4], DevBuf& counts,
                     DevBuf& scan_tmp, hipStream_t st);
// The same over at most n_cap records whose count is read on the device
// (*n_dev), with no host round trip; the sorted words are left where the
// last pass put them (where[k]).  Buffers must already hold n_cap records.
lp_status radix_sort_device_count(const SortSpec& spec, int64_t n_cap, const unsigned long long* n_dev,
                                  DevBuf tmp[4], DevBuf& counts, DevBuf& scan_tmp, hipStream_t st,
                                  uint32_t** where);

// ---------------------------------------------------------------------------
// The per-source query with every count on the device (predict.hip), for
// replay as a HIP graph: reserve() sizes the workspace for a shape (moved:
// some buffer was reallocated, so launches recorded earlier are stale; new
// dense slabs are cleared on st, before anything recorded later runs there);
// enqueue() issues the whole call with no host round trip, allocation or
// memset, reading the query count and sources from pinned host_in
// (query_device_in_bytes: u32 count at 0, sources from byte 64) and writing
// status words and results to pinned host_out (query_device_out_bytes:
// results from byte 512: c and score, qcap * kq each, then the per-query
// counts); status() checks the status words after the stream has finished.
// ---------------------------------------------------------------------------
struct QueryShape {
  int m;
  int64_t L;
  int32_t kq;
  float s_th;
  uint32_t qcap;   // sources per call, at most
  uint64_t pcap;   // two-hop paths (candidates) per call, at most
  unsigned slabs;  // dense accumulators (sources above the LDS capacity, overflowing tables)
  unsigned rounds; // rounds of `slabs` such sources (more of them: run again on the host-driven path)
};
size_t query_device_in_bytes(uint32_t qcap);
// a digest of the workspace buffers (and dense slabs) that recorded launches
// point into: recorded launches are stale once it changes
uint64_t query_device_layout(const Workspace& w);
size_t query_device_out_bytes(uint32_t qcap, int32_t kq);
lp_status query_device_reserve(lp_graph* g, Workspace& w, const QueryShape& sh, bool* moved, hipStream_t st);
lp_status query_device_enqueue(lp_graph* g, Workspace& w, const QueryShape& sh, const void* host_in,
                               void* host_out, hipStream_t st);
// LP_ERR_OUT_OF_MEMORY (with no message) when the call exceeded the shape's
// capacities and must run again on the host-driven path; *candidates: the
// candidates the call emitted
lp_status query_device_status(const void* host_out, const QueryShape& sh, uint32_t nq,
                              uint64_t* candidates);

int num_cus();
// total memory of the current device in bytes (cached on first use)
size_t device_memory();

// default upper bounds of T = U + d_a for the buckets tiny .. mid3: the
// table sizes the kernels are built for (a tuning may only lower them)
constexpr int64_t kBucketMaxDefault[5] = {32, 256, 1024, 2048, 4096};

}  // namespace lp

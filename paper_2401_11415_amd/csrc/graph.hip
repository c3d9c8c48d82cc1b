// graph.hip - building the resident graph on the device.
//
// Input: a simple undirected graph in CSR form (Section 3: G(V, E); Section
// 5.1: 32-bit vertex ids).  The resident form relabels vertices by ascending
// (degree, original id), so that the explored intermediates of a source (degree
// <= L_H, Section 4.2.1) form a prefix of its row.  For the prediction
// orientation (Algorithm 1, scanEdges skips c <= a) it keeps a compacted
// "two-hop arc list" per source: the arcs a->b whose row b holds some id > a,
// with the position where that part of row b starts and the running total of
// its lengths, so that the number of wedges a source owns for any hub limit is
// one binary search away and no work is spent on arcs without wedges.
#include <algorithm>
#include <cstring>

#include "lp_common.h"

namespace lp {

enum : uint32_t {
  kErrOffsets = 1,
  kErrIndexRange = 2,
  kErrSelfLoop = 4,
  kErrUnsorted = 8,
  kErrAsymmetric = 16,
};

constexpr int kThreads = 256;

static inline unsigned blocks_for(int64_t n, int per = kThreads) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 0x7FFFFFFF) b = 0x7FFFFFFF;
  return (unsigned)b;
}

__global__ void check_offsets_kernel(const int64_t* __restrict__ off, int64_t n, int64_t arcs,
                                     uint32_t* err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  bool bad = false;
  if (i == 0 && off[0] != 0) bad = true;
  if (i == n && off[n] != arcs) bad = true;
  if (i < n && off[i] > off[i + 1]) bad = true;
  if (off[i] < 0 || off[i] > arcs) bad = true;
  if (bad) atomicOr(err, kErrOffsets);
}

__global__ void check_indices_kernel(const int32_t* __restrict__ idx, int64_t arcs, int64_t n,
                                     uint32_t* err) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < arcs;
       e += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = idx[e];
    if (v < 0 || (int64_t)v >= n) atomicOr(err, kErrIndexRange);
  }
}

// per row: no self loop, strictly ascending (no duplicates)
__global__ void check_rows_kernel(const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                                  int64_t n, uint32_t* err) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  uint32_t bad = 0;
  for (int64_t e = off[r]; e < off[r + 1]; e++) {
    if (idx[e] == r) bad |= kErrSelfLoop;
    if (e > off[r] && idx[e] <= idx[e - 1]) bad |= kErrUnsorted;
  }
  if (bad) atomicOr(err, bad);
}

__global__ void degree_kernel(const int64_t* __restrict__ off, int64_t n, uint32_t* __restrict__ deg,
                              uint32_t* __restrict__ ids) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  deg[v] = (uint32_t)(off[v + 1] - off[v]);
  ids[v] = (uint32_t)v;
}

// perm (sorted ids) -> rank, and degrees in the new order (deg_new[n] = 0)
__global__ void relabel_kernel(const uint32_t* __restrict__ perm, const int64_t* __restrict__ off,
                               int64_t n, uint32_t* __restrict__ rank,
                               uint32_t* __restrict__ deg_new) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == n) {
    deg_new[n] = 0;
    return;
  }
  uint32_t old = perm[i];
  rank[old] = (uint32_t)i;
  deg_new[i] = (uint32_t)(off[old + 1] - off[old]);
}

// Arc p of the new layout, in new-row order v: (rank of its old neighbour, v).
// A stable sort by the first word then yields every row sorted by column.
__global__ void gather_arcs_kernel(const uint32_t* __restrict__ off_new, int64_t n,
                                   const uint32_t* __restrict__ perm,
                                   const int64_t* __restrict__ off_old,
                                   const int32_t* __restrict__ idx_old,
                                   const uint32_t* __restrict__ rank, int64_t arcs,
                                   uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < arcs;
       p += (int64_t)gridDim.x * blockDim.x) {
    // row v: last v with off_new[v] <= p
    int64_t lo = 0, hi = n;  // answer in [0, n)
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (off_new[mid] <= (uint64_t)p) lo = mid; else hi = mid;
    }
    const int64_t v = lo;
    const int64_t j = p - off_new[v];
    const int32_t u = idx_old[off_old[perm[v]] + j];
    key[p] = rank[u];
    val[p] = (uint32_t)v;
  }
}

// first position in adj[lo, hi) whose value is > x
__device__ inline uint32_t upper_bound_u32(const uint32_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                           uint32_t x) {
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ inline uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                           uint32_t x) {
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// arc p = (a -> b): start of {c in row b : c > a}; its length; symmetry check
__global__ void suffix_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                              const uint32_t* __restrict__ arow, int64_t arcs, int validate,
                              uint32_t* __restrict__ sufstart, uint32_t* __restrict__ suflen,
                              uint32_t* err) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < arcs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t a = arow[p], b = adj[p];
    const uint32_t lo = off[b], hi = off[b + 1];
    const uint32_t s = upper_bound_u32(adj, lo, hi, a);
    sufstart[p] = s;
    suflen[p] = hi - s;
    if (validate && (s == lo || adj[s - 1] != a)) atomicOr(err, kErrAsymmetric);
  }
}

// psum[p] = inclusive prefix of suflen within row a
__global__ void row_prefix_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ arow,
                                  const uint32_t* __restrict__ suflen,
                                  const uint64_t* __restrict__ incl, int64_t arcs,
                                  uint32_t* __restrict__ psum) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < arcs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s0 = off[arow[p]];
    const uint64_t row_base = incl[s0] - suflen[s0];
    psum[p] = (uint32_t)(incl[p] - row_base);
  }
}

__global__ void nz_flag_kernel(const uint32_t* __restrict__ suflen, int64_t arcs,
                               uint32_t* __restrict__ flag) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= arcs;
       p += (int64_t)gridDim.x * blockDim.x)
    flag[p] = (p < arcs && suflen[p] > 0) ? 1u : 0u;
}

__global__ void nz_compact_kernel(const uint32_t* __restrict__ pos, const uint32_t* __restrict__ suflen,
                                  const uint32_t* __restrict__ adj, const uint32_t* __restrict__ sufstart,
                                  const uint32_t* __restrict__ psum, const uint32_t* __restrict__ deg,
                                  int64_t arcs, uint32_t* __restrict__ hdeg,
                                  uint32_t* __restrict__ hstart, uint32_t* __restrict__ hpsum) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < arcs;
       p += (int64_t)gridDim.x * blockDim.x) {
    if (suflen[p] == 0) continue;
    const uint32_t q = pos[p];
    hdeg[q] = deg[adj[p]];
    hstart[q] = sufstart[p];
    hpsum[q] = psum[p];
  }
}

__global__ void nz_offsets_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ pos,
                                  int64_t n, uint32_t* __restrict__ hoff) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a <= n) hoff[a] = pos[off[a]];
}

__global__ void below_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                             int64_t n, uint32_t* __restrict__ below) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  below[a] = lower_bound_u32(adj, off[a], off[a + 1], (uint32_t)a) - off[a];
}

static int bits_for(uint64_t v) {
  int b = 0;
  while (b < 32 && (v >> b) != 0) b++;
  return b < 1 ? 1 : b;
}

uint32_t hub_start(const lp_graph* g, int64_t L) {
  if (L < 0) return 0;
  if (L >= g->max_deg) return (uint32_t)g->n;
  auto it = std::upper_bound(g->host_deg.begin(), g->host_deg.end(), (uint32_t)L);
  return (uint32_t)(it - g->host_deg.begin());
}

static void free_graph_arrays(lp_graph* g) {
  uint32_t** arrs[] = {&g->off, &g->adj, &g->hoff, &g->hdeg, &g->hstart, &g->hpsum,
                       &g->deg, &g->below, &g->perm, &g->rank, &g->deg_first};
  for (auto p : arrs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
}

struct TempBufs {
  DevBuf b[16];
  ~TempBufs() {
    for (auto& x : b) x.release();
  }
};

lp_status build_graph(int64_t n, const int64_t* offsets, const int32_t* indices, uint32_t flags,
                      lp_graph* g) {
  hipStream_t st = nullptr;
  LP_HIP(hipStreamCreate(&st));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } guard{st};
  TempBufs t;
  DevBuf& d_off_old = t.b[0];
  DevBuf& d_idx_old = t.b[1];
  DevBuf& d_err = t.b[2];
  DevBuf& d_ids = t.b[3];
  DevBuf& d_degold = t.b[4];
  DevBuf& d_key = t.b[5];
  DevBuf& d_val = t.b[6];
  DevBuf& d_suflen = t.b[7];
  DevBuf& d_incl = t.b[8];
  DevBuf sort_tmp[4];
  DevBuf counts, scan_tmp;
  struct Rel {
    DevBuf* b[6];
    ~Rel() {
      for (auto x : b) x->release();
    }
  } rel{{&sort_tmp[0], &sort_tmp[1], &sort_tmp[2], &sort_tmp[3], &counts, &scan_tmp}};

  LP_TRY(d_off_old.ensure((size_t)(n + 1) * 8));
  LP_HIP(hipMemcpyAsync(d_off_old.p, offsets, (size_t)(n + 1) * 8, hipMemcpyDefault, st));
  int64_t arcs = 0;
  LP_HIP(hipMemcpyAsync(&arcs, d_off_old.as<int64_t>() + n, 8, hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  if (arcs < 0 || arcs >= (int64_t)UINT32_MAX)
    return set_error(LP_ERR_INVALID_GRAPH, "offsets[n] = %lld arcs is outside [0, 2^32 - 1)",
                     (long long)arcs);
  LP_TRY(d_err.ensure(256));
  LP_HIP(hipMemsetAsync(d_err.p, 0, 4, st));
  uint32_t* err = d_err.as<uint32_t>();
  hipLaunchKernelGGL(check_offsets_kernel, dim3(blocks_for(n + 1)), dim3(kThreads), 0, st,
                     d_off_old.as<int64_t>(), n, arcs, err);
  LP_HIP(hipGetLastError());
  LP_TRY(d_idx_old.ensure((size_t)std::max<int64_t>(arcs, 1) * 4));
  if (arcs > 0) {
    LP_HIP(hipMemcpyAsync(d_idx_old.p, indices, (size_t)arcs * 4, hipMemcpyDefault, st));
    hipLaunchKernelGGL(check_indices_kernel, dim3(std::min<unsigned>(blocks_for(arcs), 65536u)),
                       dim3(kThreads), 0, st, d_idx_old.as<int32_t>(), arcs, n, err);
    LP_HIP(hipGetLastError());
  }
  uint32_t herr = 0;
  LP_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  if (herr & kErrOffsets) return set_error(LP_ERR_INVALID_GRAPH, "offsets are not a valid CSR prefix");
  if (herr & kErrIndexRange) return set_error(LP_ERR_INVALID_GRAPH, "an index is outside [0, n)");
  const bool validate = (flags & LP_VALIDATE) != 0;
  if (validate && n > 0) {
    hipLaunchKernelGGL(check_rows_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                       d_off_old.as<int64_t>(), d_idx_old.as<int32_t>(), n, err);
    LP_HIP(hipGetLastError());
  }

  // resident arrays
  size_t nb = (size_t)(n + 1) * 4, ab = (size_t)std::max<int64_t>(arcs, 1) * 4;
  LP_HIP(hipMalloc((void**)&g->off, nb));
  LP_HIP(hipMalloc((void**)&g->deg, nb));
  LP_HIP(hipMalloc((void**)&g->below, nb));
  LP_HIP(hipMalloc((void**)&g->perm, nb));
  LP_HIP(hipMalloc((void**)&g->rank, nb));
  LP_HIP(hipMalloc((void**)&g->adj, ab));
  LP_HIP(hipMalloc((void**)&g->hoff, nb));
  g->device_bytes = (int64_t)(6 * nb + ab);

  // 1. degrees and the (degree, id) order
  LP_TRY(d_ids.ensure(nb));
  LP_TRY(d_degold.ensure(nb));
  if (n > 0) {
    hipLaunchKernelGGL(degree_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st,
                       d_off_old.as<int64_t>(), n, d_degold.as<uint32_t>(), d_ids.as<uint32_t>());
    LP_HIP(hipGetLastError());
    SortSpec sp{};
    sp.w[0] = d_degold.as<uint32_t>();
    sp.w[1] = d_ids.as<uint32_t>();
    sp.nwords = 2;
    sp.nkeys = 1;
    sp.key_bits[0] = 32;
    // bits actually used by degrees: arcs bound every degree
    sp.key_bits[0] = bits_for((uint64_t)arcs);
    LP_TRY(radix_sort(sp, n, sort_tmp, counts, scan_tmp, st));
    LP_HIP(hipMemcpyAsync(g->perm, d_ids.p, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  }
  hipLaunchKernelGGL(relabel_kernel, dim3(blocks_for(n + 1)), dim3(kThreads), 0, st, g->perm,
                     d_off_old.as<int64_t>(), n, g->rank, g->deg);
  LP_HIP(hipGetLastError());
  LP_TRY(scan_exclusive_u32(g->deg, g->off, n + 1, scan_tmp, st));

  // 2. arcs in the new labelling, rows sorted
  if (arcs > 0) {
    LP_TRY(d_key.ensure(ab));
    LP_TRY(d_val.ensure(ab));
    unsigned gb = std::min<unsigned>(blocks_for(arcs), 65536u);
    hipLaunchKernelGGL(gather_arcs_kernel, dim3(gb), dim3(kThreads), 0, st, g->off, n, g->perm,
                       d_off_old.as<int64_t>(), d_idx_old.as<int32_t>(), g->rank, arcs,
                       d_key.as<uint32_t>(), d_val.as<uint32_t>());
    LP_HIP(hipGetLastError());
    SortSpec sp{};
    sp.w[0] = d_key.as<uint32_t>();
    sp.w[1] = d_val.as<uint32_t>();
    sp.nwords = 2;
    sp.nkeys = 1;
    sp.key_bits[0] = bits_for((uint64_t)(n > 0 ? n - 1 : 0));
    LP_TRY(radix_sort(sp, arcs, sort_tmp, counts, scan_tmp, st));
    LP_HIP(hipMemcpyAsync(g->adj, d_val.p, (size_t)arcs * 4, hipMemcpyDeviceToDevice, st));
    const uint32_t* arow = d_key.as<uint32_t>();

    // 3. suffix starts, lengths and per-row running totals
    DevBuf& d_sufstart = t.b[9];
    DevBuf& d_psum = t.b[10];
    DevBuf& d_pos = t.b[11];
    LP_TRY(d_suflen.ensure(ab));
    LP_TRY(d_sufstart.ensure(ab));
    LP_TRY(d_psum.ensure(ab));
    hipLaunchKernelGGL(suffix_kernel, dim3(gb), dim3(kThreads), 0, st, g->off, g->adj, arow, arcs,
                       validate ? 1 : 0, d_sufstart.as<uint32_t>(), d_suflen.as<uint32_t>(), err);
    LP_HIP(hipGetLastError());
    LP_TRY(d_incl.ensure((size_t)arcs * 8));
    LP_TRY(scan_inclusive_u32_u64(d_suflen.as<uint32_t>(), d_incl.as<uint64_t>(), arcs, scan_tmp, st));
    hipLaunchKernelGGL(row_prefix_kernel, dim3(gb), dim3(kThreads), 0, st, g->off, arow,
                       d_suflen.as<uint32_t>(), d_incl.as<uint64_t>(), arcs, d_psum.as<uint32_t>());
    LP_HIP(hipGetLastError());
    // 4. keep the arcs with a non-empty suffix (order preserved)
    LP_TRY(d_pos.ensure((size_t)(arcs + 1) * 8));
    uint32_t* flag = d_pos.as<uint32_t>();
    uint32_t* pos = flag + (arcs + 1);
    hipLaunchKernelGGL(nz_flag_kernel, dim3(gb), dim3(kThreads), 0, st, d_suflen.as<uint32_t>(), arcs,
                       flag);
    LP_HIP(hipGetLastError());
    LP_TRY(scan_exclusive_u32(flag, pos, arcs + 1, scan_tmp, st));
    uint32_t H = 0;
    LP_HIP(hipMemcpyAsync(&H, pos + arcs, 4, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    size_t hbytes = (size_t)std::max<uint32_t>(H, 1) * 4;
    LP_HIP(hipMalloc((void**)&g->hdeg, hbytes));
    LP_HIP(hipMalloc((void**)&g->hstart, hbytes));
    LP_HIP(hipMalloc((void**)&g->hpsum, hbytes));
    g->device_bytes += (int64_t)(3 * hbytes);
    g->harcs = H;
    hipLaunchKernelGGL(nz_compact_kernel, dim3(gb), dim3(kThreads), 0, st, pos,
                       d_suflen.as<uint32_t>(), g->adj, d_sufstart.as<uint32_t>(),
                       d_psum.as<uint32_t>(), g->deg, arcs, g->hdeg, g->hstart, g->hpsum);
    LP_HIP(hipGetLastError());
    hipLaunchKernelGGL(nz_offsets_kernel, dim3(blocks_for(n + 1)), dim3(kThreads), 0, st, g->off, pos,
                       n, g->hoff);
    LP_HIP(hipGetLastError());
  } else {
    LP_HIP(hipMemsetAsync(g->hoff, 0, nb, st));
    LP_HIP(hipMalloc((void**)&g->hdeg, 4));
    LP_HIP(hipMalloc((void**)&g->hstart, 4));
    LP_HIP(hipMalloc((void**)&g->hpsum, 4));
  }
  if (n > 0) {
    hipLaunchKernelGGL(below_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st, g->off, g->adj, n,
                       g->below);
    LP_HIP(hipGetLastError());
  }
  g->host_deg.resize((size_t)n);
  if (n > 0)
    LP_HIP(hipMemcpyAsync(g->host_deg.data(), g->deg, (size_t)n * 4, hipMemcpyDeviceToHost, st));
  LP_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  if (herr & kErrSelfLoop) return set_error(LP_ERR_INVALID_GRAPH, "the graph has a self-loop");
  if (herr & kErrUnsorted)
    return set_error(LP_ERR_INVALID_GRAPH, "a row is not strictly ascending (unsorted or duplicate)");
  if (herr & kErrAsymmetric) return set_error(LP_ERR_INVALID_GRAPH, "the graph is not symmetric");
  g->n = n;
  g->arcs = arcs;
  g->max_deg = n > 0 ? g->host_deg[(size_t)n - 1] : 0;
  // degree -> first new id of at least that degree (ids are in degree order),
  // for degrees up to deg_cap; scoring uses it to bound d_c from an id alone
  {
    const uint32_t cap = (uint32_t)std::min<int64_t>(g->max_deg + 1, 65536);
    std::vector<uint32_t> first((size_t)cap + 1);
    for (uint32_t d = 0; d <= cap; d++)
      first[d] = (uint32_t)(std::lower_bound(g->host_deg.begin(), g->host_deg.end(), d) - g->host_deg.begin());
    LP_HIP(hipMalloc((void**)&g->deg_first, first.size() * 4));
    LP_HIP(hipMemcpy(g->deg_first, first.data(), first.size() * 4, hipMemcpyHostToDevice));
    g->deg_cap = cap;
    g->device_bytes += (int64_t)(first.size() * 4);
  }
  // AA / RA fixed point: a sum of at most max_deg terms, each <= 1/ln 2 < 1.45,
  // must stay below 2^63.
  int shift = 44;
  while (shift > 16 && (double)(g->max_deg + 1) * 1.45 * std::ldexp(1.0, shift) >= std::ldexp(1.0, 62))
    shift--;
  g->fixed_shift = shift;
  return LP_OK;
}

void release_workspace(Workspace& w) {
  DevBuf* all[] = {&w.cnt, &w.wedges, &w.lists, &w.counters, &w.stats, &w.cand_s, &w.cand_a,
                   &w.cand_c, &w.tmp_s[0], &w.tmp_s[1], &w.tmp_a[0], &w.tmp_a[1], &w.tmp_c[0],
                   &w.tmp_c[1], &w.hist, &w.sel_state, &w.sort_tmp[0], &w.sort_tmp[1],
                   &w.sort_tmp[2], &w.sort_tmp[3], &w.sort_counts, &w.scan_tmp, &w.global_tab, &w.unfit, &w.kept, &w.q_src,
                   &w.q_cnt, &w.q_wedges, &w.q_rows, &w.q_out, &w.m_graph, &w.m_gid,
                   &w.m_lists, &w.spa_meta};
  for (auto b : all) b->release();
  w.host_stats.release();
  w.m_checked.clear();
  for (int i = 0; i < Workspace::kSide; i++) {
    if (w.side[i]) (void)hipStreamDestroy(w.side[i]);
    if (w.join[i]) (void)hipEventDestroy(w.join[i]);
    w.side[i] = nullptr;
    w.join[i] = nullptr;
  }
  if (w.fork) (void)hipEventDestroy(w.fork);
  w.fork = nullptr;
  for (auto& e : w.clock_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  for (auto& e : w.timer_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
}

void destroy_graph(lp_graph* g) {
  free_graph_arrays(g);
  release_workspace(g->ws);
}

}  // namespace lp

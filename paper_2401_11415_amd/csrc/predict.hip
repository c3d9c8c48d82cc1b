// predict.hip - the hot path: per-source two-hop accumulation (IBase / DLH),
// first-order exclusion, fused scoring, candidate filtering and top-k.
//
// Method (Sahu, arXiv 2401.11415, Section 4.1 and 4.2, Algorithm 1): for
// every source a, every explored intermediate b in Gamma_a (d_b <= L_H) and
// every c in Gamma_b with c > a, count the path a-b-c under key c (or add the
// AA / RA weight of b); drop keys that are first-order neighbours of a; score
// each remaining key; keep the best N_P pairs overall.
//
// GPU design (gfx950, wave64):
//  * plan: for each source its explored arcs (a prefix of its two-hop arc
//    list, since intermediates are ordered by degree) and its exact wedge
//    count U(a); sources go to seven buckets by T = U + (first-order
//    neighbours after a).
//  * accumulation: small sources run in batches (48 or 8 per 256-lane
//    workgroup, 4 per 512 lanes) that share one LDS hash table keyed by
//    (position in the batch, c); larger ones get a whole workgroup (256, 512
//    or 1024 lanes) and a table sized by a bound on their distinct keys,
//    split into hash partitions when it exceeds the LDS; sources whose keys
//    exceed the LDS capacity use a dense accumulator in global memory.  A
//    window decoder turns 64 consecutive flat wedge indices into (arc,
//    position) pairs with one ballot, so lanes read consecutive ids of the
//    same neighbour list (coalesced).
//  * count tables (CN ... LHN) hold (count << 32 | key) per 64-bit slot; AA /
//    RA tables hold key and fixed-point sum in one 64-bit slot when the
//    per-source precision bound allows, else 12-byte slots.
//  * with a top-k threshold, the normalised measures bound the degree (hence
//    the id) of any candidate that can still pass: wedges to ids at or above
//    that cutoff are loaded but not inserted.  AA / RA sources whose arc
//    weights sum below the threshold are dropped before their batch runs.
//  * scoring is fused into the table sweep; survivors of S_th and of a key
//    threshold tau are appended with one atomic per wave.
//  * top-k: MSD radix select over the 96-bit key (score bits, ~a, ~c), then a
//    stable LSD radix sort of the k winners.  tau is estimated from a sampled
//    subset of sources so that only about k candidates are ever written.
#include <algorithm>
#include <cmath>
#include <cstring>

#include <memory>

#include "kernels.h"

namespace lp {

// ---------------------------------------------------------------------------
// Plan: per source, its explored arcs and wedge count, written as a record
// into the list of its scheduling bucket.
// ---------------------------------------------------------------------------

enum : int {
  kBucketTiny = 0,   // T <= 32:      48 sources per 256-lane workgroup
  kBucketSmall = 1,  // T <= 256:     8 sources per workgroup
  kBucketMid1 = 2,   // T <= 1024:    4 sources per 512-lane workgroup (12-byte tables: 2 per 256)
  kBucketMid2 = 3,   // T <= 2048:    256 lanes per source
  kBucketMid3 = 4,   // T <= 4096:    512 lanes per source
  kBucketLarge = 5,  // T <= cap:     1024 lanes, hash partitions
  kBucketHuge = 6,   // T >  cap:     dense accumulator in global memory (unless few keys: large)
  kBuckets = 7
};

// One source as the accumulation kernels see it (32 bytes, one load).
struct SrcRec {
  uint32_t a;    // relabelled id
  uint32_t key;  // predict: original id; query: query index
  uint32_t h0;   // first explored arc (two-hop list for predict, adj for query)
  uint32_t na;   // explored arcs
  uint32_t U;    // wedges (predict: exact; query: upper bound)
  uint32_t x0;   // first-order neighbours to exclude: adj[x0, x1)
  uint32_t x1;
  uint32_t da;   // degree
};

struct PlanOut {
  unsigned long long wedges;
  unsigned long long sources;
  uint32_t count[kBuckets];
  uint32_t bad_source;
};

__device__ inline uint32_t lower_bound_dev(const uint32_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                           uint32_t x) {
  while (lo < hi) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Bucket of a source with U wedges and T = U + (first-order neighbours to
// exclude) table entries at most; sources without wedges have no candidates.
// Upper bounds of T = U + d_a per bucket: tiny .. mid3, then the LDS cap
// (larger sources take the global path).  The defaults are the table sizes
// the kernels are built for; a tuning may only lower the first five.
struct BucketCuts {
  uint32_t t[kBucketHuge];
};

// keys: a bound of the source's distinct keys (prediction orientation: the
// ids above it, which can be far fewer than its wedges); a source above the
// LDS capacity by wedges still takes an LDS table, in a few partitions, when
// its keys fit the capacity and its wedges are at most 4 times it
__device__ inline int bucket_of(uint32_t U, uint32_t T, const BucketCuts& cut, uint32_t keys = 0xFFFFFFFFu) {
  if (U == 0) return -1;
  if (T > cut.t[kBucketLarge])
    return keys <= cut.t[kBucketLarge] && T / 4 <= cut.t[kBucketLarge] ? kBucketLarge : kBucketHuge;
#pragma unroll
  for (int b = kBucketTiny; b < kBucketLarge; b++)
    if (T <= cut.t[b]) return b;
  return kBucketLarge;
}

constexpr int kPlanItems = 4;  // sources per thread of the plan kernel

// Bucket a tile of 256 * kPlanItems sources with one global atomic per
// (workgroup, bucket); records land in lists[bucket * stride + position].
// A source's explored arcs are the prefix of its two-hop arcs whose
// intermediate has degree < hub_deg (= L + 1, clamped); the list ascends by
// intermediate, hence by degree.
__global__ __launch_bounds__(256) void plan_kernel(GView g, uint32_t hub_deg, BucketCuts cuts,
                                                   SrcRec* __restrict__ lists,
                                                   PlanOut* __restrict__ out) {
  __shared__ uint32_t wtot[kBuckets][4];
  __shared__ uint32_t bbase[kBuckets];
  __shared__ unsigned long long red_w[4], red_s[4];
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const uint64_t tile = (uint64_t)blockIdx.x * 256 * kPlanItems;
  uint8_t bk[kPlanItems];
  uint32_t nb[kBuckets] = {};
  unsigned long long w_sum = 0, s_sum = 0;
  // explored prefix of every item's two-hop arcs: the binary searches of a
  // thread's items run in lockstep, so each step has kPlanItems independent
  // loads in flight instead of one dependent chain per item
  uint32_t lo[kPlanItems], hi[kPlanItems], na[kPlanItems];
#pragma unroll
  for (int j = 0; j < kPlanItems; j++) {
    const uint64_t a = tile + (uint64_t)j * 256 + threadIdx.x;
    lo[j] = hi[j] = 0;
    if (a < g.n) {
      lo[j] = g.hoff[a];
      hi[j] = g.hoff[a + 1];
    }
    na[j] = lo[j];  // row start, until the search ends
  }
  for (;;) {
    bool more = false;
#pragma unroll
    for (int j = 0; j < kPlanItems; j++) more = more | (lo[j] < hi[j]);
    if (!more) break;
    // an item whose search has ended reads entry 0, which exists: some item
    // of this thread still has arcs
    uint32_t v[kPlanItems];
#pragma unroll
    for (int j = 0; j < kPlanItems; j++) v[j] = g.hdeg[lo[j] < hi[j] ? lo[j] + ((hi[j] - lo[j]) >> 1) : 0u];
#pragma unroll
    for (int j = 0; j < kPlanItems; j++) {
      if (lo[j] < hi[j]) {
        const uint32_t mid = lo[j] + ((hi[j] - lo[j]) >> 1);
        if (v[j] < hub_deg) lo[j] = mid + 1;
        else hi[j] = mid;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kPlanItems; j++) na[j] = lo[j] - na[j];
#pragma unroll
  for (int j = 0; j < kPlanItems; j++) {
    const uint64_t a = tile + (uint64_t)j * 256 + threadIdx.x;
    bk[j] = 0xFF;
    if (a < g.n) {
      const uint32_t h0 = g.hoff[a], h1 = g.hoff[a + 1];
      uint32_t U = 0, T = 0;
      if (h1 > h0) {
        const uint32_t k = na[j];
        U = k ? g.hpsum[h0 + k - 1] : 0u;
        // the bucket follows the work (wedges), not the key bound: a source
        // with many wedges but few reachable keys still needs many lanes
        const uint64_t t = (uint64_t)U + (g.off[a + 1] - g.off[a] - g.below[a]);
        T = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
      }
      const uint32_t room = (uint32_t)(g.n - 1 - a);  // keys lie in (a, n)
      const int b = bucket_of(U, T, cuts, T < room ? T : room);
      if (b >= 0) {
        bk[j] = (uint8_t)b;
        nb[b]++;
        w_sum += U;
        s_sum += 1;
      }
    }
  }
  uint32_t excl[kBuckets];
#pragma unroll
  for (int b = 0; b < kBuckets; b++) {
    uint32_t x = nb[b];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    excl[b] = x - nb[b];
    if (lane == 63) wtot[b][wid] = x;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    w_sum += __shfl_xor(w_sum, o);
    s_sum += __shfl_xor(s_sum, o);
  }
  if (lane == 0) {
    red_w[wid] = w_sum;
    red_s[wid] = s_sum;
  }
  __syncthreads();
  if (threadIdx.x < kBuckets) {
    const int b = threadIdx.x;
    const uint32_t t = wtot[b][0] + wtot[b][1] + wtot[b][2] + wtot[b][3];
    bbase[b] = t ? atomicAdd(&out->count[b], t) : 0u;
  }
  if (threadIdx.x == 64) {
    const unsigned long long ws = red_w[0] + red_w[1] + red_w[2] + red_w[3];
    const unsigned long long ss = red_s[0] + red_s[1] + red_s[2] + red_s[3];
    if (ss) {
      atomicAdd(&out->wedges, ws);
      atomicAdd(&out->sources, ss);
    }
  }
  __syncthreads();
  uint32_t pos[kBuckets];
#pragma unroll
  for (int b = 0; b < kBuckets; b++) {
    pos[b] = bbase[b] + excl[b];
    for (int w = 0; w < wid; w++) pos[b] += wtot[b][w];
  }
#pragma unroll
  for (int j = 0; j < kPlanItems; j++) {
    if (bk[j] == 0xFF) continue;
    const uint32_t a = (uint32_t)(tile + (uint64_t)j * 256 + threadIdx.x);
    // second read of the row start: cheap (cached)
    const uint32_t h0 = g.hoff[a];
    const uint32_t k = na[j];
    SrcRec r;
    r.a = a;
    r.key = g.perm[a];
    r.h0 = h0;
    r.na = k;
    r.U = g.hpsum[h0 + k - 1];
    const uint32_t e0 = g.off[a];
    r.x1 = g.off[a + 1];
    r.x0 = e0 + g.below[a];
    r.da = r.x1 - e0;
#pragma unroll
    for (int b = 0; b < kBuckets; b++)
      if (bk[j] == b) lists[(uint64_t)b * g.n + pos[b]++] = r;
  }
}

// query: map sources to new ids, explored prefix of the row and an upper
// bound of the wedges (all of Gamma_b for explored b), one workgroup per query
__global__ __launch_bounds__(256) void query_plan_kernel(GView g, uint32_t hub_start,
                                                         BucketCuts cuts,
                                                         const int32_t* __restrict__ src,
                                                         const uint32_t* __restrict__ rank,
                                                         uint32_t nq, SrcRec* __restrict__ lists,
                                                         PlanOut* __restrict__ out,
                                                         const uint32_t* __restrict__ nq_dev) {
  __shared__ unsigned long long part[4];
  // nq: the stride of the bucket lists; with nq_dev the queries themselves
  // are counted on the device (at most nq)
  const uint32_t nreq = nq_dev ? min(*nq_dev, nq) : nq;
  for (uint32_t q = blockIdx.x; q < nreq; q += gridDim.x) {
    const int32_t so = src[q];
    const bool ok = so >= 0 && (uint32_t)so < g.n;
    if (!ok && threadIdx.x == 0) atomicOr(&out->bad_source, 1u);
    const uint32_t s = ok ? rank[so] : 0u;
    const uint32_t e0 = g.off[s], e1 = g.off[s + 1];
    const uint32_t k = ok ? lower_bound_dev(g.adj, e0, e1, hub_start) - e0 : 0u;
    unsigned long long sum = 0;
    for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) sum += g.deg[g.adj[e0 + j]];
    for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
    if (lane_id() == 0) part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long tot = part[0] + part[1] + part[2] + part[3];
      const uint32_t U = tot > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)tot;
      const uint64_t t = (uint64_t)U + (e1 - e0);
      const int b = bucket_of(U, t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t, cuts);
      if (b >= 0) {
        SrcRec r;
        r.a = s;
        r.key = q;
        r.h0 = e0;
        r.na = k;
        r.U = U;
        r.x0 = e0;
        r.x1 = e1;
        r.da = e1 - e0;
        const uint32_t pos = atomicAdd(&out->count[b], 1u);
        lists[(uint64_t)b * nq + pos] = r;
        atomicAdd(&out->wedges, (unsigned long long)U);
        atomicAdd(&out->sources, 1ull);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Work lists: which records a launch processes.
//   phase 0: all; 1: every stride-th (the sample); 2: the others.
// ---------------------------------------------------------------------------

struct WorkList {
  const SrcRec* list;
  uint32_t count;
  uint32_t stride;
  int phase;
  const uint32_t* count_dev = nullptr;  // if set: phase 0, count read on the device
};

__device__ inline uint32_t work_count(const WorkList& w) {
  if (w.count_dev) return *w.count_dev;
  if (w.phase == 0 || w.stride <= 1) return w.phase == 2 ? 0u : w.count;
  const uint32_t ns = (w.count + w.stride - 1) / w.stride;
  return w.phase == 1 ? ns : w.count - ns;
}

__device__ inline uint32_t work_index(const WorkList& w, uint32_t i) {
  if (w.phase == 0 || w.stride <= 1) return i;
  if (w.phase == 1) return i * w.stride;
  const uint32_t s1 = w.stride - 1;
  return (i / s1) * w.stride + (i % s1) + 1;
}

__device__ inline SrcRec load_rec(const WorkList& w, uint32_t i) { return w.list[work_index(w, i)]; }

// A record that the whole wave works on, held in scalar registers.
__device__ inline SrcRec uniform_rec(const SrcRec& r) {
  return SrcRec{uniform(r.a), uniform(r.key), uniform(r.h0), uniform(r.na),
                uniform(r.U),   uniform(r.x0),  uniform(r.x1), uniform(r.da)};
}

// Load the chunk of explored arcs [cb, cb + G) of source s into the group
// scratch: flat index of its first wedge (excl), position in adj of its first
// c (start), weight; the chunk covers flat wedges [*lo, *hi).
// Weights are fixed point with wshift fraction bits, lifted by wlift bits
// (packed tables keep the key below the sum).
template <int G, bool kQuery, bool kW>
__device__ inline void load_chunk(const GView& g, const Emit& E, const SrcRec& s, uint32_t cb,
                                  uint32_t* s_excl, uint32_t* s_start, uint64_t* s_w,
                                  uint32_t* scan_tmp, uint32_t* lo, uint32_t* hi, int wshift,
                                  int wlift = 0) {
  const int gl = threadIdx.x & (G - 1);
  const uint32_t j = cb + gl;
  const bool valid = j < s.na;
  const uint32_t e = s.h0 + j;
  uint32_t start = 0, len = 0;
  uint64_t w = 0;
  if (kQuery) {
    if (valid) {
      const uint32_t b = g.adj[e];
      start = g.off[b];
      len = g.off[b + 1] - start;
      if (kW) w = weight_of(E.measure, len, wshift) << wlift;
    }
    uint32_t total;
    const uint32_t ex = group_exclusive_scan<G>(len, scan_tmp, &total);
    s_excl[gl] = valid ? ex : kEmpty32;
    *lo = 0;
    *hi = uniform(total);
  } else {
    uint32_t ex = kEmpty32;
    if (valid) {
      start = g.hstart[e];
      ex = j == 0 ? 0u : g.hpsum[e - 1];
      if (kW) w = weight_of(E.measure, g.hdeg[e], wshift) << wlift;
    }
    s_excl[gl] = ex;
    const uint32_t last = (cb + G < s.na ? cb + G : s.na) - 1;
    *lo = uniform(cb == 0 ? 0u : g.hpsum[s.h0 + cb - 1]);
    *hi = uniform(g.hpsum[s.h0 + last]);
  }
  s_start[gl] = start;
  if (kW) s_w[gl] = w;
}

// Linear probing slows down sharply as a table fills, so a table that fits
// its workgroup's slots in one partition takes up to a spread times its key
// bound, in halves: kSpreadHalves[batched][weighted].  Sums spread most
// (load <= 1/3): on the AA / RA workloads nearly every wedge is a new key, so
// their tables come close to the bound.  R-MAT count tables hold about one
// key per 1.3 wedges, so a wider table mostly lengthens the sweep: per-source
// tables take 2x, batch tables keep 1.5x.  (Chung-Lu 8M RA at L = 256: 47.0
// ms per call with 1.5x everywhere, 39.7 with 2x, 38.5 with 3x; R-MAT-22 JC
// mid1 batches 1.83, 1.87, 2.0 ms; its per-source kernels gain with 2x.)
constexpr uint32_t kSpreadHalves[2][2] = {{4, 6}, {3, 6}};

// Table geometry of a source with at most U keys: P hash partitions (each
// loaded at most 2/3), S slots each.
__device__ inline void table_geometry(uint32_t U, uint32_t slots, uint32_t* P, uint32_t* S,
                                      uint32_t spread_halves) {
  const uint64_t need = ((uint64_t)U * 3 + 1) / 2;
  if (need <= slots) {
    *P = 1;
    const uint64_t roomy = std::min<uint64_t>((uint64_t)U * spread_halves / 2, slots);
    *S = roomy < 16 ? 16u : (uint32_t)roomy;
    return;
  }
  uint32_t p = (uint32_t)((need + slots - 1) / slots);
  if (p < 1) p = 1;
  const uint64_t per = ((uint64_t)U + p - 1) / p;
  uint64_t s = (per * 3 + 1) / 2;
  if (s < 16) s = 16;
  if (s > slots) s = slots;
  *P = p;
  *S = (uint32_t)s;
}

// partition of a key (range reduction of its Fibonacci hash)
__device__ inline uint32_t key_part(uint32_t c, uint32_t P) {
  return (uint32_t)(((uint64_t)(c * kHashMul) * P) >> 32);
}

// ---------------------------------------------------------------------------
// Shared pieces of the accumulation kernels
// ---------------------------------------------------------------------------

constexpr int kWin = 4;  // windows of 64 wedges a wave decodes per round

// Walk one wave's slice of a chunk's flat wedge range [lo, hi): the range is
// cut into NWG slices of whole windows, one per wave of the group (wig =
// wave's index in the group).  Per round of kWin windows, fn(c, arc, v) gets
// each lane's wedges c (kEmpty32 where v is false) and their arcs.  Rounds
// are software-pipelined: the next round is decoded and its wedge loads are
// in flight while fn works on the current one.
template <int NWG, int GA>
struct WalkRound {
  uint32_t arc[kWin], c[kWin];
  bool v[kWin];
  // decode the round starting at base (j: arc holding base, advanced) and
  // issue its wedge loads
  __device__ void start(const GView& g, const uint32_t* excl, const uint32_t* start_of, uint32_t narcs,
                        uint8_t* mark, uint32_t base, uint32_t f1, uint32_t& j) {
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t idx[kWin];
#pragma unroll
    for (int u = 0; u < kWin; u++) {
      const uint32_t b = base + 64u * u;
      arc[u] = 0;
      v[u] = false;
      idx[u] = 0;
      if (b < f1) {
        arc[u] = decode_window(excl, narcs, mark, b, j);
        v[u] = b + lane < f1;
        if (v[u]) idx[u] = start_of[arc[u]] + (b + lane - excl[arc[u]]);
      }
    }
    // every lane loads (idx 0 where the lane has no wedge), so the loads need
    // no branches; the ids are masked where the round is consumed, so that
    // nothing waits for the loads before then
#pragma unroll
    for (int u = 0; u < kWin; u++) c[u] = g.adj[idx[u]];
  }
};

template <int NWG, int GA, typename Fn>
__device__ inline void walk_chunk(const GView& g, const uint32_t* excl, const uint32_t* start,
                                  uint32_t narcs, uint32_t lo, uint32_t hi, int wig, uint8_t* mark,
                                  Fn&& fn) {
  const uint64_t per = ((uint64_t)(hi - lo) + NWG - 1) / NWG;
  const uint64_t q = (per + 63) & ~63ull;
  const uint64_t f0l = (uint64_t)lo + (uint64_t)wig * q;
  if (f0l >= hi) return;
  const uint32_t f0 = (uint32_t)f0l;
  const uint32_t f1 = (uint32_t)(f0l + q < (uint64_t)hi ? f0l + q : (uint64_t)hi);
  uint32_t j = uniform((uint32_t)seg_search<GA>(excl, f0));
  // Two rounds in turn, so that no register copy of loaded ids (which would
  // wait for the loads) sits between issuing a round and consuming it.  A
  // round past the slice's end is still issued (no valid window, loads of
  // entry 0): a conditional issue would make the compiler wait for every
  // load in flight where the two paths meet.
  constexpr uint32_t R = 64 * kWin;
  WalkRound<NWG, GA> A, B;
  A.start(g, excl, start, narcs, mark, f0, f1, j);
  for (uint32_t base = f0; base < f1; base += 2 * R) {
    B.start(g, excl, start, narcs, mark, base + R, f1, j);
#pragma unroll
    for (int u = 0; u < kWin; u++) A.c[u] = A.v[u] ? A.c[u] : kEmpty32;
    fn(A.c, A.arc, A.v);
    if (base + R >= f1) break;
    A.start(g, excl, start, narcs, mark, base + 2 * R, f1, j);
#pragma unroll
    for (int u = 0; u < kWin; u++) B.c[u] = B.v[u] ? B.c[u] : kEmpty32;
    fn(B.c, B.arc, B.v);
  }
}

// ---------------------------------------------------------------------------
// LDS-table accumulation: groups of G lanes (G a multiple of 64; WGS / G
// groups per workgroup), one source per group at a time, up to SLOTS slots.
// ---------------------------------------------------------------------------

template <int WGS, int G, int SLOTS, int TM, int STAGE, bool kQ = false>
struct LdsTab {
  static constexpr int NG = WGS / G;
  static constexpr int NW = WGS / 64;
  static constexpr bool kW = TM != kTabCount;
  static constexpr bool kSplit = TM == kTabSplit;
  uint64_t tab[kSplit ? 1 : NG * SLOTS];
  uint32_t keys[kSplit ? NG * SLOTS : 1];
  uint64_t vals[kSplit ? NG * SLOTS : 1];
  uint32_t excl[NG][G];
  uint32_t start[NG][G];
  uint64_t w[kW ? NG : 1][kW ? G : 1];
  uint32_t scan_tmp[G > 64 ? G / 64 : 1];
  int ovf[NG][2];
  uint8_t mark[NW][64];
  uint32_t rt_key[NW][64];
  uint32_t rt_h[NW][64];
  uint64_t rt_w[kW ? NW : 1][64];
  // weighted queries: a histogram of the group's sums and its floor
  uint32_t qhist[kQ ? NG : 1][kQ ? kSumBins : 1];
  uint64_t qfloor[kQ ? NG : 1];
  uint32_t st_c[NW][STAGE];
  uint32_t st_h[NW][STAGE];
  uint32_t st_w2[kW ? NW : 1][kW ? STAGE : 1];
  uint32_t st_k[NW][STAGE];
  uint32_t st_d[NW][STAGE];
  uint32_t so_s[NW][64];
  uint32_t so_a[NW][64];
  uint32_t so_c[NW][64];
};

// kSampled: the same kernel instantiated separately for the sampling pass,
// so that profiles and per-launch statistics keep the two passes apart
// Packed tables ask for at most 128 VGPRs (four waves per SIMD): without the
// bound the compiler gives their kernels 130-150, and then a 512-lane
// workgroup, or four 256-lane ones, no longer share a CU with another.  (The
// count kernels stay below 128 by themselves and run slower under the bound.)
template <int WGS, int G, int SLOTS, int TM, bool kQuery, int STAGE, bool kSampled>
__global__ __launch_bounds__(WGS, TM == kTabPacked ? 4 : 1) void acc_lds_kernel(GView g, Emit E, WorkList wl) {
  static_assert(G % 64 == 0 && (G == 64 || G == WGS), "groups are whole waves");
  static_assert(STAGE >= 64, "a stage holds at least one wave of entries");
  static_assert(!(TM == kTabPacked && kQuery), "packed sums are for the prediction orientation");
  constexpr int NG = WGS / G;
  constexpr bool kW = TM != kTabCount;
  constexpr bool kSplit = TM == kTabSplit;
  constexpr bool kPacked = TM == kTabPacked;
  __shared__ LdsTab<WGS, G, SLOTS, TM, STAGE, kW && kQuery> L;
  const int grp = (int)uniform(threadIdx.x / G);
  const int gl = threadIdx.x & (G - 1);
  const int wv = threadIdx.x >> 6;
  uint64_t* tab = L.tab + (kSplit ? 0 : grp * SLOTS);
  uint32_t* keys = L.keys + (kSplit ? grp * SLOTS : 0);
  uint64_t* vals = L.vals + (kSplit ? grp * SLOTS : 0);
  // packed tables: the key is the id itself
  const int kb = kPacked ? E.pk_idbits : 32;
  const uint32_t kmask = kPacked ? (uint32_t)((1ull << kb) - 1) : kEmpty32;
  const uint64_t empty = kPacked ? (uint64_t)kmask : kSlotEmpty;
  uint32_t* s_excl = L.excl[grp];
  uint32_t* s_start = L.start[grp];
  uint64_t* s_w = kW ? L.w[grp] : nullptr;
  uint8_t* mark = L.mark[wv];
  mark[lane_id()] = 0;
  wave_fence();
  Stage SG{L.st_c[wv], L.st_h[wv], kW ? L.st_w2[wv] : nullptr, L.st_k[wv], L.st_d[wv],
           (uint32_t)STAGE, L.so_s[wv], L.so_a[wv], L.so_c[wv], 64u};
  Retry<kW> RT{L.rt_key[wv], L.rt_h[wv], kW ? L.rt_w[wv] : nullptr};
  FpAcc fa;
  WorkAcc wk;
  const uint32_t total = uniform(work_count(wl));
  // slots [0, clean) of the group's table are empty: every sweep empties the
  // slots it reads, so only growth beyond the largest table so far is cleared
  uint32_t clean = 0;
  // The group meets at two barriers per source (and chunk of arcs): after the
  // chunk scratch is loaded and after the last table update.  The sweep of
  // one source runs into the next source's first barrier, which is safe: the
  // next source clears only slots beyond the swept ones, and its first table
  // update follows that barrier.  The overflow flag alternates between two
  // words so that resetting one cannot race a late reader.
  uint32_t par = 0;
  const uint32_t step = gridDim.x * NG;
  uint32_t i = blockIdx.x * NG + grp;
  SrcRec nxt{};
  if (i < total) nxt = load_rec(wl, i);
  for (; i < total; i += step) {
    const SrcRec s = uniform_rec(nxt);
    if (i + step < total) nxt = load_rec(wl, i + step);  // in flight during this source
    // first batch of first-order ids, in flight during the accumulation (from
    // the group's last wave on, which has the lightest share of the wedges)
    const uint32_t xe = s.x0 + (G - 1 - gl);
    const uint32_t xb = xe < s.x1 ? g.adj[xe] : kEmpty32;
    // the source's threshold (its graph's, when several graphs run at once)
    const uint32_t ts_bits = E.fp_mode ? 0u : uniform((kQuery ? E.tau : tau_of(E, s.key))[0]);
    const uint64_t wmin = kW ? min_wsum(E.measure, ts_bits, E.shift) : 1ull;
    const double lo = E.fp_mode ? 0.0 : pass_edge(ts_bits, E.s_th);
    const uint32_t hmin = kW ? 1u : min_count(E.measure, ts_bits, s.da, !kQuery);
    const uint32_t cut1 = kW ? 0xFFFFFFFFu : uniform(id_cutoff(E.measure, 1, s.da, lo, g, !kQuery));
    const uint32_t cut2 = kW ? 0xFFFFFFFFu : uniform(id_cutoff(E.measure, 2, s.da, lo, g, !kQuery));
    // no count exceeds the explored arcs: ids at or above the cutoff for that
    // count cannot pass, so their wedges are not accumulated at all
    const uint32_t cut_all = (kW || kQuery) ? 0xFFFFFFFFu
                                            : uniform(id_cutoff(E.measure, s.na < s.da ? s.na : s.da, s.da,
                                                                lo, g, true));
    // every key lies in (a, min(n, cut_all)) in the prediction orientation,
    // which bounds the distinct keys far below the wedges for high-rank sources
    uint32_t keys_max = s.U + (s.x1 - s.x0);
    if (!kQuery) {
      const uint32_t top = cut_all < g.n ? cut_all : g.n;
      const uint32_t room = top > s.a + 1 ? top - s.a - 1 : 0u;
      keys_max = room < keys_max ? room : keys_max;
    }
    uint32_t P, S;
    table_geometry(keys_max, SLOTS, &P, &S, kSpreadHalves[0][kW ? 1 : 0]);
    // packed sums: a source whose sums may not fit is handed over whole
    if (kPacked && !packed_fits(E.measure, s.na, kb, E.shift)) {
      if (gl == 0) hand_unfit(E, s);
      continue;
    }
    bool handed = false;
    for (uint32_t pass = 0; pass < P; pass++) {
      if (S > clean) {
        for (uint32_t t = clean + gl; t < S; t += G) {
          if (kSplit) {
            keys[t] = kEmpty32;
            vals[t] = 0;
          } else {
            tab[t] = empty;
          }
        }
        clean = S;
      }
      par ^= 1u;
      if (gl == 0) L.ovf[grp][par] = 0;
      bool full = false;
      for (uint32_t cb = 0; cb < s.na; cb += G) {
        uint32_t lo, hi;
        if (cb > 0) group_sync<G>();  // every wave is done with the previous chunk
        load_chunk<G, kQuery, kW>(g, E, s, cb, s_excl, s_start, s_w, L.scan_tmp, &lo, &hi, E.shift,
                                  kPacked ? kb : 0);
        group_sync<G>();
        const uint32_t narcs = s.na - cb < (uint32_t)G ? s.na - cb : (uint32_t)G;
        walk_chunk<G / 64, G>(g, s_excl, s_start, narcs, lo, hi, (int)uniform(gl >> 6), mark,
                              [&](const uint32_t (&c)[kWin], const uint32_t (&arc)[kWin],
                                  const bool (&v)[kWin]) {
          uint32_t key[kWin];
          uint64_t inc[kWin];
#pragma unroll
          for (int u = 0; u < kWin; u++) {
            bool live = v[u] & (c[u] < cut_all);
            if (kQuery) live = live & (c[u] != s.a);
            if (P > 1) live = live & (key_part(c[u], P) == pass);
            key[u] = live ? c[u] : kEmpty32;
            inc[u] = kW ? s_w[arc[u]] : kSlotOne;
          }
          if constexpr (kSplit) {
#pragma unroll
            for (int u = 0; u < kWin; u++)
              full = full | !tab_insert<TM>(tab, keys, vals, S, key[u], key_slot(key[u], S), inc[u], RT, kmask);
          } else {
            full = full | !tab_insert_k<TM, kWin>(tab, S, key, inc, RT, kmask);
          }
        });
      }
      // first-order neighbours are not candidates: they enter flagged
      for (uint32_t e0 = s.x0; e0 < s.x1; e0 += G) {
        const uint32_t e = e0 + (G - 1 - gl);
        uint32_t b = e0 == s.x0 ? xb : (e < s.x1 ? g.adj[e] : kEmpty32);
        if (b >= cut_all) b = kEmpty32;  // no wedge key at or above the cutoff exists
        if (P > 1 && b != kEmpty32 && key_part(b, P) != pass) b = kEmpty32;
        const bool ok = tab_insert<TM>(tab, keys, vals, S, b, key_slot(b, S),
                                       kW ? kBlocked64W : kBlocked64, RT, kmask);
        full = full | !ok;
      }
      full = full | !retry_drain<TM>(tab, keys, vals, S, RT, kmask);
      if (full) L.ovf[grp][par] = 1;
      group_sync<G>();
      if (L.ovf[grp][par]) {
        // the table filled up: hand the rest of this source to the global path
        clean = 0;
        if (gl == 0) {
          const uint32_t slot = atomicAdd(E.ovf_count, 1u);
          if (slot < E.ovf_cap) {
            static_cast<SrcRec*>(E.ovf_rec)[slot] = s;
            E.ovf[slot] = pass | (P << 8);
          } else {
            atomicOr(E.err, kErrOvfList);
          }
        }
        group_sync<G>();
        handed = true;
        break;
      }
      // a weighted query needs only the k_q best sums of the source: the
      // floor of a histogram of this partition's sums bounds them below
      uint64_t wmin_q = wmin;
      if constexpr (kW && kQuery) {
        if (E.kq > 0 && S > 4 * E.kq) {
          uint32_t* qh = L.qhist[grp];
          for (uint32_t b = gl; b < kSumBins; b += G) qh[b] = 0;
          group_sync<G>();
          for (uint32_t t = gl; t < S; t += G) {
            const uint64_t v = vals[t];
            if (keys[t] != kEmpty32 && v != 0 && (v >> 63) == 0) atomicAdd(&qh[sum_bin(v)], 1u);
          }
          group_sync<G>();
          if (gl < 64) {
            const uint64_t f = sum_floor_wave(qh, E.kq);
            if (gl == 0) L.qfloor[grp] = f;
          }
          group_sync<G>();
          const uint64_t f = uniform64(L.qfloor[grp]);
          wmin_q = f > wmin ? f : wmin;
        }
      }
      // stage every key of this partition that can still reach tau, and
      // leave the table empty for the next source
      for (uint32_t t0 = 0; t0 < S; t0 += G) {
        const uint32_t t = t0 + gl;
        const uint32_t tc = t < S ? t : 0u;
        uint32_t c, h = 0;
        uint64_t wsum = 0;
        bool cand, ok;
        if (kSplit) {
          c = keys[tc];
          wsum = vals[tc];
          if (t < S) {
            keys[t] = kEmpty32;
            vals[t] = 0;
          }
          cand = t < S && c != kEmpty32 && (wsum >> 63) == 0;
          ok = cand && wsum >= wmin_q;
        } else if (kPacked) {
          const uint64_t v = tab[tc];
          if (t < S) tab[t] = empty;
          c = (uint32_t)v & kmask;
          cand = t < S && c != kmask && (v >> 63) == 0;
          wsum = cand ? packed_sum(v, kb) : 0ull;
          ok = cand && wsum >= wmin_q;
        } else {
          const uint64_t v = tab[tc];
          if (t < S) tab[t] = kSlotEmpty;
          c = (uint32_t)v;
          h = (uint32_t)(v >> 32);
          cand = t < S && c != kEmpty32 && (h & kBlocked) == 0;
          ok = cand && h >= hmin && !(h == 1 && c >= cut1) && !(h == 2 && c >= cut2);
        }
        wk.v[4] += cand ? 1u : 0u;
        stage_add<kQuery, kW>(E, g, SG, ok, c, h, wsum, s.key, s.da, fa);
      }
    }
    if (!handed && gl == 0) wk.source(s.da, s.na, s.U);
  }
  stage_drain<kQuery, kW>(E, g, SG, fa);
  flush_fp(E, fa);
  flush_work(E, wk);
}

// ---------------------------------------------------------------------------
// Batched LDS accumulation for small sources (prediction orientation): one
// workgroup takes B consecutive sources of a bucket and accumulates all their
// wedges into one table keyed by (position in the batch, c), so the batch pays
// the dependent global round trips (records, arcs, wedges, first-order rows)
// once instead of once per source.  A key packs the position in the batch
// above the id bits, so B bounds the vertex count (BatchKey::kMaxN).
// ---------------------------------------------------------------------------

template <int B>
struct BatchKey {
  static_assert(B >= 1 && B <= 64, "batch fits in one wave");
  static constexpr int kSrcBits = B <= 2 ? 1 : B <= 4 ? 2 : B <= 8 ? 3 : B <= 16 ? 4 : B <= 32 ? 5 : 6;
  static constexpr int kIdBits = 32 - kSrcBits;
  static constexpr uint32_t kIdMask = (1u << kIdBits) - 1;
  // largest vertex count whose keys all stay below the empty key
  static constexpr uint64_t kMaxN =
      (1ull << kIdBits) < 0xFFFFFFFFull - ((uint64_t)(B - 1) << kIdBits)
          ? (1ull << kIdBits)
          : 0xFFFFFFFFull - ((uint64_t)(B - 1) << kIdBits);
};
static_assert(BatchKey<48>::kMaxN == (1ull << 26) && BatchKey<32>::kMaxN == (1ull << 27) - 1 &&
                  BatchKey<2>::kMaxN == (1ull << 31) - 1,
              "batch key ranges");

template <int WGS, int B, int SLOTS, int TM, int STAGE>
struct BatchTab {
  static constexpr int NW = WGS / 64;
  static constexpr bool kW = TM != kTabCount;
  static constexpr bool kSplit = TM == kTabSplit;
  uint64_t tab[kSplit ? 1 : SLOTS];
  uint32_t keys[kSplit ? SLOTS : 1];
  uint64_t vals[kSplit ? SLOTS : 1];
  uint32_t excl[WGS];
  uint32_t start[WGS];
  uint32_t srcof[WGS];
  uint64_t w[kW ? WGS : 1];
  SrcRec rec[B];
  uint32_t arcoff[B + 1];  // prefix of explored arcs
  uint32_t wedoff[B + 1];  // prefix of wedges
  uint32_t xoff[B + 1];    // prefix of first-order neighbours to exclude
  uint32_t keys_max;       // bound of the batch's distinct keys
  uint32_t hmin[B];
  uint64_t wmin[kW ? B : 1];
  uint8_t fits[TM == kTabPacked ? B : 1];  // packed sums: the source's sums fit its slots
  uint32_t cut[B][2];
  uint32_t cut_all[B];
  int ovf;
  uint8_t mark[NW][64];
  uint32_t rt_key[NW][64];
  uint32_t rt_h[NW][64];
  uint64_t rt_w[kW ? NW : 1][64];
  uint32_t st_c[NW][STAGE];
  uint32_t st_h[NW][STAGE];
  uint32_t st_w2[kW ? NW : 1][kW ? STAGE : 1];
  uint32_t st_k[NW][STAGE];
  uint32_t st_d[NW][STAGE];
  uint32_t so_s[NW][64];
  uint32_t so_a[NW][64];
  uint32_t so_c[NW][64];
};

// last index i in [0, B) with off[i] <= q (off non-decreasing, off[0] == 0 <= q)
template <int B>
__device__ inline int batch_search(const uint32_t* off, uint32_t q) {
  int lo = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1)
    if (step < B && lo + step < B && off[lo + step] <= q) lo += step;
  return lo;
}

template <int WGS, int B, int SLOTS, int TM, int STAGE, bool kSampled>
__global__ __launch_bounds__(WGS, TM == kTabPacked ? 4 : 1) void acc_batch_kernel(GView g, Emit E, WorkList wl) {
  using KB = BatchKey<B>;
  constexpr int NW = WGS / 64;
  constexpr bool kW = TM != kTabCount;
  constexpr bool kSplit = TM == kTabSplit;
  constexpr bool kPacked = TM == kTabPacked;
  __shared__ BatchTab<WGS, B, SLOTS, TM, STAGE> L;
  // a key is (position in the batch, id): count and split tables keep the
  // position in the top bits of 32; packed tables right above the id bits
  const int ib = kPacked ? E.pk_idbits : KB::kIdBits;
  const uint32_t imask = kPacked ? (uint32_t)((1ull << ib) - 1) : KB::kIdMask;
  const int kb = kPacked ? ib + KB::kSrcBits : 32;
  const uint32_t kmask = kPacked ? (uint32_t)((1ull << kb) - 1) : kEmpty32;
  const uint64_t empty = kPacked ? (uint64_t)kmask : kSlotEmpty;
  const int tid = threadIdx.x;
  const int wv = tid >> 6;
  uint8_t* mark = L.mark[wv];
  mark[lane_id()] = 0;
  wave_fence();
  Stage SG{L.st_c[wv], L.st_h[wv], kW ? L.st_w2[wv] : nullptr, L.st_k[wv], L.st_d[wv],
           (uint32_t)STAGE, L.so_s[wv], L.so_a[wv], L.so_c[wv], 64u};
  Retry<kW> RT{L.rt_key[wv], L.rt_h[wv], kW ? L.rt_w[wv] : nullptr};
  FpAcc fa;
  WorkAcc wk;
  const uint32_t total = uniform(work_count(wl));
  const uint32_t nbatch = (total + B - 1) / B;
  uint32_t clean = 0;  // slots [0, clean) of the table are empty
  // the first wave keeps the next batch's records in flight
  SrcRec nrec{};
  if (tid < B && blockIdx.x * B + tid < total) nrec = load_rec(wl, blockIdx.x * B + tid);
  for (uint32_t bi = blockIdx.x; bi < nbatch; bi += gridDim.x) {
    const uint32_t i0 = bi * B;
    const uint32_t nb = total - i0 < (uint32_t)B ? total - i0 : (uint32_t)B;
    // records and their prefix sums (first wave); the id cutoffs are loaded
    // here and published after the accumulation, off the critical path
    uint32_t cut0 = 0xFFFFFFFFu, cut1 = 0xFFFFFFFFu, cutv = 0xFFFFFFFFu;
    if (tid < 64) {
      SrcRec r{};
      uint32_t na = 0, U = 0, nx = 0, km = 0;
      if (tid < (int)nb) {
        r = nrec;
        na = r.na;
        U = r.U;
        nx = r.x1 - r.x0;
        if (kPacked) {
          // packed sums: a source whose sums may not fit is handed over
          // whole and takes no part in the batch
          const bool fits = packed_fits(E.measure, na, kb, E.shift);
          L.fits[tid] = fits ? 1 : 0;
          if (!fits) {
            hand_unfit(E, r);
            na = U = nx = 0;
          }
        }
        L.rec[tid] = r;
        // the source's threshold (its graph's, when several graphs run at once)
        const uint32_t ts_bits = E.fp_mode ? 0u : tau_of(E, r.key)[0];
        const double lo = E.fp_mode ? 0.0 : pass_edge(ts_bits, E.s_th);
        L.hmin[tid] = kW ? 1u : min_count(E.measure, ts_bits, r.da, true);
        if (kW) L.wmin[tid] = min_wsum(E.measure, ts_bits, E.shift);
        if (!kW) {
          cut0 = id_cutoff(E.measure, 1, r.da, lo, g, true);
          cut1 = id_cutoff(E.measure, 2, r.da, lo, g, true);
          // no count exceeds the explored arcs: wedges to ids at or above the
          // cutoff for that count are not accumulated
          cutv = id_cutoff(E.measure, r.na < r.da ? r.na : r.da, r.da, lo, g, true);
          L.cut_all[tid] = cutv;
        }
        // keys lie in (a, min(n, cutoff))
        const uint32_t top = cutv < g.n ? cutv : g.n;
        const uint32_t room = top > r.a + 1 ? top - r.a - 1 : 0u;
        km = U + nx < room ? U + nx : room;
      }
      const uint32_t inext = i0 + gridDim.x * B + tid;
      if (tid < B && inext < total) nrec = load_rec(wl, inext);
      uint32_t xa = na, xu = U, xx = nx;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t ya = __shfl_up(xa, o, 64), yu = __shfl_up(xu, o, 64), yx = __shfl_up(xx, o, 64);
        km += __shfl_xor(km, o, 64);
        if (tid >= o) {
          xa += ya;
          xu += yu;
          xx += yx;
        }
      }
      if (tid == 0) L.keys_max = km;
      if (tid < B) {
        L.arcoff[tid] = xa - na;
        L.wedoff[tid] = xu - U;
        L.xoff[tid] = xx - nx;
      }
      if (tid == B - 1) {
        L.arcoff[B] = xa;
        L.wedoff[B] = xu;
        L.xoff[B] = xx;
      }
      if (tid == 0) L.ovf = 0;
    }
    __syncthreads();
    const uint32_t NA = uniform(L.arcoff[B]), NX = uniform(L.xoff[B]);
    // the batch's table, spread like a source's (table_geometry) and capped
    // at the kernel's slots
    uint32_t S = (uint32_t)std::min<uint64_t>(
        (uint64_t)uniform(L.keys_max) * kSpreadHalves[1][kW ? 1 : 0] / 2, SLOTS);
    if (S < 16) S = 16;
    // first batch of first-order keys, in flight during the accumulation
    uint32_t xkey = kEmpty32;
    if ((uint32_t)(WGS - 1 - tid) < NX) {
      const uint32_t xq = (uint32_t)(WGS - 1 - tid);
      const uint32_t xi = (uint32_t)batch_search<B>(L.xoff, xq);
      xkey = (xi << ib) | g.adj[L.rec[xi].x0 + (xq - L.xoff[xi])];
    }
    if (S > clean) {
      for (uint32_t t = clean + tid; t < S; t += WGS) {
        if (kSplit) {
          L.keys[t] = kEmpty32;
          L.vals[t] = 0;
        } else {
          L.tab[t] = empty;
        }
      }
      clean = S;
    }
    bool full = false;
    for (uint32_t cb = 0; cb < NA; cb += WGS) {
      if (cb > 0) __syncthreads();  // every wave is done with the previous chunk
      const uint32_t q = cb + tid;
      const bool qin = q < NA;
      const uint32_t qc = qin ? q : cb;
      const uint32_t si = (uint32_t)batch_search<B>(L.arcoff, qc);
      const uint32_t local = qc - L.arcoff[si];
      const uint32_t e = L.rec[si].h0 + local;
      const uint32_t start = g.hstart[e];
      const uint32_t prev = local == 0 ? 0u : g.hpsum[e - 1];
      uint64_t w = 0;
      if (kSplit) w = weight_of(E.measure, g.hdeg[e], E.shift);
      if (kPacked && qin) w = weight_of(E.measure, g.hdeg[e], E.shift) << kb;
      L.excl[tid] = qin ? L.wedoff[si] + prev : kEmpty32;
      L.start[tid] = start;
      L.srcof[tid] = si;
      if (kW) L.w[tid] = w;
      // flat wedge range of this chunk
      const uint32_t qlast = (cb + WGS < NA ? cb + WGS : NA) - 1;
      const uint32_t sl = (uint32_t)batch_search<B>(L.arcoff, qlast);
      const uint32_t hi = uniform(L.wedoff[sl] + g.hpsum[L.rec[sl].h0 + (qlast - L.arcoff[sl])]);
      __syncthreads();
      const uint32_t lo = uniform(L.excl[0]);
      const uint32_t narcs = NA - cb < (uint32_t)WGS ? NA - cb : (uint32_t)WGS;
      walk_chunk<NW, WGS>(g, L.excl, L.start, narcs, lo, hi, (int)uniform(wv), mark,
                          [&](const uint32_t (&c)[kWin], const uint32_t (&arc)[kWin],
                              const bool (&v)[kWin]) {
        uint32_t key[kWin];
        uint64_t inc[kWin];
#pragma unroll
        for (int u = 0; u < kWin; u++) {
          const uint32_t si = L.srcof[arc[u]];
          // no count exceeds the explored arcs: wedges to ids at or above a
          // source's cutoff for that count cannot pass and are not accumulated
          const bool live = kW ? v[u] : (v[u] && c[u] < L.cut_all[si]);
          key[u] = live ? (si << ib) | (c[u] & imask) : kEmpty32;
          inc[u] = kW ? L.w[arc[u]] : kSlotOne;
        }
        if constexpr (kSplit) {
#pragma unroll
          for (int u = 0; u < kWin; u++)
            full = full | !tab_insert<TM>(L.tab, L.keys, L.vals, S, key[u], key_slot(key[u], S), inc[u], RT, kmask);
        } else {
          full = full | !tab_insert_k<TM, kWin>(L.tab, S, key, inc, RT, kmask);
        }
      });
    }
    if (tid < (int)nb) {
      L.cut[tid][0] = cut0;
      L.cut[tid][1] = cut1;
    }
    // first-order neighbours are not candidates: they enter flagged (from the
    // last wave on, which has the lightest share of the wedges)
    for (uint32_t x0 = 0; x0 < NX; x0 += WGS) {
      const uint32_t x = x0 + (WGS - 1 - tid);
      uint32_t key = x0 == 0 ? xkey : kEmpty32;
      if (x0 != 0 && x < NX) {
        const uint32_t i = (uint32_t)batch_search<B>(L.xoff, x);
        key = (i << ib) | g.adj[L.rec[i].x0 + (x - L.xoff[i])];
      }
      // no wedge key at or above the source's cutoff exists
      if (!kW && key != kEmpty32 && (key & imask) >= L.cut_all[key >> ib]) key = kEmpty32;
      const bool ok = tab_insert<TM>(L.tab, L.keys, L.vals, S, key, key_slot(key, S),
                                     kW ? kBlocked64W : kBlocked64, RT, kmask);
      full = full | !ok;
    }
    full = full | !retry_drain<TM>(L.tab, L.keys, L.vals, S, RT, kmask);
    if (full) L.ovf = 1;
    __syncthreads();
    if (L.ovf) {
      // a full table: every source of the batch goes to the global path whole
      clean = 0;
      if (tid < (int)nb) {
        const uint32_t slot = atomicAdd(E.ovf_count, 1u);
        if (slot < E.ovf_cap) {
          static_cast<SrcRec*>(E.ovf_rec)[slot] = L.rec[tid];
          E.ovf[slot] = 0u | (1u << 8);
        } else {
          atomicOr(E.err, kErrOvfList);
        }
      }
      __syncthreads();
      continue;
    }
    if (tid < (int)nb && (!kPacked || L.fits[tid])) wk.source(L.rec[tid].da, L.rec[tid].na, L.rec[tid].U);
    // stage every key that can still reach tau
    for (uint32_t t0 = 0; t0 < S; t0 += WGS) {
      const uint32_t t = t0 + tid;
      const uint32_t tc = t < S ? t : 0u;
      uint32_t key, h = 0;
      uint64_t wsum = 0;
      bool ok;
      if (kSplit) {
        key = L.keys[tc];
        wsum = L.vals[tc];
        if (t < S) {
          L.keys[t] = kEmpty32;
          L.vals[t] = 0;
        }
        ok = t < S && key != kEmpty32 && (wsum >> 63) == 0;
        wk.v[4] += ok ? 1u : 0u;
        ok = ok && wsum >= L.wmin[ok ? key >> ib : 0u];
      } else if (kPacked) {
        const uint64_t v = L.tab[tc];
        if (t < S) L.tab[t] = empty;
        key = (uint32_t)v & kmask;
        ok = t < S && key != kmask && (v >> 63) == 0;
        wk.v[4] += ok ? 1u : 0u;
        const uint32_t i = ok ? key >> ib : 0u;
        wsum = ok ? packed_sum(v, kb) : 0ull;
        ok = ok && wsum >= L.wmin[i];
      } else {
        const uint64_t v = L.tab[tc];
        if (t < S) L.tab[t] = kSlotEmpty;
        key = (uint32_t)v;
        h = (uint32_t)(v >> 32);
        ok = t < S && key != kEmpty32 && (h & kBlocked) == 0;
        wk.v[4] += ok ? 1u : 0u;
      }
      const uint32_t i = ok ? key >> ib : 0u;
      if (!kW) {
        const uint32_t c = key & imask;
        ok = ok && h >= L.hmin[i] && !(h == 1 && c >= L.cut[i][0]) && !(h == 2 && c >= L.cut[i][1]);
      }
      stage_add<false, kW>(E, g, SG, ok, key & imask, h, wsum, L.rec[i].key, L.rec[i].da, fa);
    }
    __syncthreads();
  }
  stage_drain<false, kW>(E, g, SG, fa);
  flush_fp(E, fa);
  flush_work(E, wk);
}

// ---------------------------------------------------------------------------
// Dense accumulator in global memory (the paper's per-thread table: a value
// per vertex plus a key list), one workgroup per source.  Used for sources
// whose wedge count exceeds the LDS capacity and for partitions handed over
// by an overflowing LDS table.
// ---------------------------------------------------------------------------

struct SpaItem {
  const uint32_t* ovf;  // if non-null: overflow entries (pass | P << 8) ...
  const SrcRec* recs;   // ... and their source records
  uint32_t ovf_begin, ovf_end;
  const uint32_t* end_dev = nullptr;  // if set: the end is read on the device (at most ovf_end)
};

constexpr int kSpaThreads = 1024;
constexpr int kSpaStage = 128;

template <bool kW, bool kQuery, bool kSampled>
__global__ __launch_bounds__(kSpaThreads) void acc_spa_kernel(GView g, Emit E, WorkList wl,
                                                              SpaItem ov, char* spa_acc,
                                                              uint32_t* spa_keys) {
  constexpr int T = kSpaThreads;
  constexpr int NW = T / 64;
  __shared__ uint32_t s_excl[T], s_start[T], scan_tmp[NW];
  __shared__ uint64_t s_w[kW ? T : 1];
  __shared__ uint32_t nkeys;
  __shared__ uint8_t s_mark[NW][64];
  __shared__ uint32_t st_c[NW][kSpaStage], st_h[NW][kSpaStage], st_k[NW][kSpaStage],
      st_d[NW][kSpaStage], st_w2[kW ? NW : 1][kW ? kSpaStage : 1];
  __shared__ uint32_t so_s[NW][64], so_a[NW][64], so_c[NW][64];
  // weighted queries: a histogram of the source's sums and its floor
  __shared__ uint32_t qh[kW && kQuery ? kSumBins : 1];
  __shared__ unsigned long long qfloor;
  const int wv = threadIdx.x >> 6;
  uint8_t* mark = s_mark[wv];
  mark[lane_id()] = 0;
  wave_fence();
  Stage SG{st_c[wv], st_h[wv], kW ? st_w2[wv] : nullptr, st_k[wv], st_d[wv], (uint32_t)kSpaStage,
           so_s[wv], so_a[wv], so_c[wv], 64u};
  // one 8-byte-per-vertex accumulator slab per workgroup, whatever the measure:
  // counts use its first half, so every slab stays zero between calls
  char* slab = spa_acc + (uint64_t)blockIdx.x * g.n * 8;
  uint32_t* H = reinterpret_cast<uint32_t*>(slab);
  unsigned long long* HW = reinterpret_cast<unsigned long long*>(slab);
  uint32_t* K = spa_keys + (uint64_t)blockIdx.x * g.n;
  FpAcc fa;
  WorkAcc wk;
  uint32_t ovf_end = ov.ovf_end;
  if (ov.ovf && ov.end_dev) ovf_end = uniform(min(*ov.end_dev, ovf_end));
  const uint32_t total = ov.ovf ? (ovf_end > ov.ovf_begin ? ovf_end - ov.ovf_begin : 0u) : uniform(work_count(wl));
  for (uint32_t i = blockIdx.x; i < total; i += gridDim.x) {
    SrcRec s;
    uint32_t p0 = 0, P = 1;
    if (ov.ovf) {
      s = uniform_rec(ov.recs[ov.ovf_begin + i]);
      const uint32_t pl = uniform(ov.ovf[ov.ovf_begin + i]);
      p0 = pl & 0xFFu;
      P = pl >> 8;
    } else {
      s = uniform_rec(load_rec(wl, i));
    }
    const uint32_t ts_bits = E.fp_mode ? 0u : uniform((kQuery ? E.tau : tau_of(E, s.key))[0]);
    const uint64_t wmin = kW ? min_wsum(E.measure, ts_bits, E.shift) : 1ull;
    const uint32_t hmin = kW ? 1u : min_count(E.measure, ts_bits, s.da, !kQuery);
    if (threadIdx.x == 0) nkeys = 0;
    __syncthreads();
    for (uint32_t cb = 0; cb < s.na; cb += T) {
      uint32_t lo, hi;
      load_chunk<T, kQuery, kW>(g, E, s, cb, s_excl, s_start, s_w, scan_tmp, &lo, &hi, E.shift);
      __syncthreads();
      const uint32_t narcs = s.na - cb < (uint32_t)T ? s.na - cb : (uint32_t)T;
      walk_chunk<NW, T>(g, s_excl, s_start, narcs, lo, hi, (int)uniform(wv), mark,
                        [&](const uint32_t (&c)[kWin], const uint32_t (&arc)[kWin],
                            const bool (&v)[kWin]) {
#pragma unroll
        for (int u = 0; u < kWin; u++) {
          if (!v[u] || (kQuery && c[u] == s.a)) continue;
          if (P > 1 && key_part(c[u], P) < p0) continue;
          bool first;
          if (kW) first = atomicAdd(&HW[c[u]], (unsigned long long)s_w[arc[u]]) == 0ull;
          else first = atomicAdd(&H[c[u]], 1u) == 0u;
          if (first)
            __hip_atomic_store(&K[atomicAdd(&nkeys, 1u)], c[u], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      });
      __syncthreads();
    }
    for (uint32_t e = s.x0 + threadIdx.x; e < s.x1; e += T) {
      const uint32_t b = g.adj[e];
      if (kW) __hip_atomic_store(&HW[b], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else __hip_atomic_store(&H[b], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __syncthreads();
    const uint32_t nk = nkeys;
    // a weighted query keeps only sums at or above the floor of its k_q-th
    // largest sum's bin (reads through the atomics' coherence point)
    uint64_t wmin_q = wmin;
    if constexpr (kW && kQuery) {
      if (E.kq > 0 && nk > 4 * E.kq) {
        for (uint32_t b = threadIdx.x; b < kSumBins; b += T) qh[b] = 0;
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < nk; t += T) {
          const uint32_t c = __hip_atomic_load(&K[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const unsigned long long v = __hip_atomic_load(&HW[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (v != 0) atomicAdd(&qh[sum_bin(v)], 1u);
        }
        __syncthreads();
        if (threadIdx.x < 64) {
          const uint64_t f = sum_floor_wave(qh, E.kq);
          if (threadIdx.x == 0) qfloor = f;
        }
        __syncthreads();
        const uint64_t f = uniform64(qfloor);
        wmin_q = f > wmin ? f : wmin;
      }
    }
    for (uint32_t t0 = 0; t0 < nk; t0 += T) {
      const uint32_t t = t0 + threadIdx.x;
      uint32_t c = 0, h = 0;
      uint64_t wsum = 0;
      bool ok = false;
      if (t < nk) {
        c = __hip_atomic_load(&K[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (kW) {
          wsum = __hip_atomic_exchange(&HW[c], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          wk.v[4] += wsum != 0 ? 1u : 0u;
          ok = wsum != 0 && wsum >= wmin_q;
        } else {
          h = __hip_atomic_exchange(&H[c], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          wk.v[4] += h != 0 ? 1u : 0u;
          ok = h != 0 && h >= hmin;
        }
      }
      stage_add<kQuery, kW>(E, g, SG, ok, c, h, wsum, s.key, s.da, fa);
    }
    if (threadIdx.x == 0) wk.source(s.da, s.na, s.U);
    __threadfence();
    __syncthreads();
  }
  stage_drain<kQuery, kW>(E, g, SG, fa);
  flush_fp(E, fa);
  flush_work(E, wk);
}

// ---------------------------------------------------------------------------
// Dense accumulation split over workgroups, for the sources above the LDS
// capacity: one workgroup per source made a hub with millions of wedges the
// tail of the whole launch.  A round takes as many sources as there are
// slabs; any workgroup takes any piece of 1024 arcs of them (atomics into the
// source's slab, first touches appended to its key list, one atomic per wave
// for the list), then the first-order entries are cleared, then pieces of
// 1024 keys are scored and emitted, which leaves every slab zero again.
// Kernel boundaries order the three steps.
// ---------------------------------------------------------------------------

struct SpaRound {
  WorkList wl;       // the bucket's work list
  uint32_t i0, n;    // the round's items: work-list positions [i0, i0 + n)
  uint32_t* poff;    // n + 1 offsets of the arc pieces ...
  uint32_t* koff;    // n + 1 offsets of the key pieces
  uint32_t* nkeys;   // n distinct keys per source (zero before the round)
  char* acc;         // slab j at acc + j * 8n
  uint32_t* keys;    // key list j at keys + j * n
  uint32_t* hist;    // query with sums: n x kSumBins bins of the sources' sums (zeroed) ...
  unsigned long long* floor_sum;  // ... and n per-source floors: the k_q-th largest sum's bin
  // if set: the work list's length, read on the device; the round then holds
  // min(n, length - i0) items (n is the slab count)
  const uint32_t* len_dev = nullptr;
};

__device__ inline uint32_t round_items(const SpaRound& R) {
  if (!R.len_dev) return R.n;
  const uint32_t len = *R.len_dev;
  const uint32_t left = len > R.i0 ? len - R.i0 : 0u;
  return left < R.n ? left : R.n;
}

constexpr uint32_t kSpaPiece = kSpaThreads;  // arcs or keys per piece

// piece offsets of a round: ceil(arcs / 1024) per source (mode 0) or
// ceil(keys / 1024) (mode 1); one workgroup
__global__ __launch_bounds__(1024) void spa_pieces_kernel(SpaRound R, int mode) {
  __shared__ uint32_t tmp[16];
  R.n = round_items(R);
  uint32_t* out = mode == 0 ? R.poff : R.koff;
  uint32_t run = 0;
  for (uint32_t j0 = 0; j0 < R.n; j0 += 1024) {
    const uint32_t j = j0 + threadIdx.x;
    uint32_t p = 0;
    if (j < R.n) {
      const uint32_t cnt = mode == 0 ? load_rec(R.wl, R.i0 + j).na : R.nkeys[j];
      p = (cnt + kSpaPiece - 1) / kSpaPiece;
    }
    uint32_t tot;
    const uint32_t ex = group_exclusive_scan<1024>(p, tmp, &tot);
    if (j < R.n) out[j] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0) out[R.n] = run;
}

// the source j of piece q: last j with off[j] <= q (off[0] = 0 <= q < off[n])
__device__ inline uint32_t spa_piece_source(const uint32_t* off, uint32_t n, uint32_t q) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= q) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <bool kW, bool kQuery, bool kSampled>
__global__ __launch_bounds__(kSpaThreads) void spa_split_acc_kernel(GView g, Emit E, SpaRound R) {
  R.n = uniform(round_items(R));
  constexpr int T = kSpaThreads;
  constexpr int NW = T / 64;
  __shared__ uint32_t s_excl[T], s_start[T], scan_tmp[NW];
  __shared__ uint64_t s_w[kW ? T : 1];
  __shared__ uint8_t s_mark[NW][64];
  const int wv = threadIdx.x >> 6;
  uint8_t* mark = s_mark[wv];
  mark[lane_id()] = 0;
  wave_fence();
  const uint32_t total = uniform(R.poff[R.n]);
  for (uint32_t q = blockIdx.x; q < total; q += gridDim.x) {
    const uint32_t j = uniform(spa_piece_source(R.poff, R.n, q));
    const SrcRec s = uniform_rec(load_rec(R.wl, R.i0 + j));
    const uint32_t cb = (q - uniform(R.poff[j])) * kSpaPiece;
    char* slab = R.acc + (uint64_t)j * g.n * 8;
    uint32_t* H = reinterpret_cast<uint32_t*>(slab);
    unsigned long long* HW = reinterpret_cast<unsigned long long*>(slab);
    uint32_t* K = R.keys + (uint64_t)j * g.n;
    uint32_t lo, hi;
    __syncthreads();  // every wave is done with the previous piece
    load_chunk<T, kQuery, kW>(g, E, s, cb, s_excl, s_start, s_w, scan_tmp, &lo, &hi, E.shift);
    __syncthreads();
    const uint32_t narcs = s.na - cb < (uint32_t)T ? s.na - cb : (uint32_t)T;
    walk_chunk<NW, T>(g, s_excl, s_start, narcs, lo, hi, (int)uniform(wv), mark,
                      [&](const uint32_t (&c)[kWin], const uint32_t (&arc)[kWin],
                          const bool (&v)[kWin]) {
#pragma unroll
      for (int u = 0; u < kWin; u++) {
        bool first = false;
        if (v[u] && !(kQuery && c[u] == s.a)) {
          if (kW) first = atomicAdd(&HW[c[u]], (unsigned long long)s_w[arc[u]]) == 0ull;
          else first = atomicAdd(&H[c[u]], 1u) == 0u;
        }
        // new keys of the wave go to the list with one atomic
        const uint64_t m = __ballot(first);
        if (m) {
          uint32_t base = 0;
          const int leader = __ffsll((unsigned long long)m) - 1;
          if (lane_id() == leader) base = atomicAdd(&R.nkeys[j], (uint32_t)__popcll(m));
          base = __shfl(base, leader);
          if (first)
            __hip_atomic_store(&K[base + (uint32_t)__popcll(m & lanemask_lt())], c[u], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    });
  }
}

// first-order neighbours are not candidates: clear their entries (one
// workgroup per source; the source's work counters are taken here)
template <bool kW, bool kQuery, bool kSampled>
__global__ __launch_bounds__(kSpaThreads) void spa_split_excl_kernel(GView g, Emit E, SpaRound R) {
  R.n = uniform(round_items(R));
  WorkAcc wk;
  for (uint32_t j = blockIdx.x; j < R.n; j += gridDim.x) {
    const SrcRec s = uniform_rec(load_rec(R.wl, R.i0 + j));
    char* slab = R.acc + (uint64_t)j * g.n * 8;
    for (uint32_t e = s.x0 + threadIdx.x; e < s.x1; e += kSpaThreads) {
      const uint32_t b = g.adj[e];
      if (kW)
        __hip_atomic_store(reinterpret_cast<unsigned long long*>(slab) + b, 0ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_store(reinterpret_cast<uint32_t*>(slab) + b, 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0) wk.source(s.da, s.na, s.U);
  }
  flush_work(E, wk);
}

// Query with sums (AA, RA): each source needs only its k_q best candidates,
// and the score grows with the sum.  A log-scale histogram of each source's
// sums gives a floor at or below its k_q-th largest sum; the sweep keeps
// only sums at or above it, so a hub no longer emits millions of candidates.
template <bool kW, bool kQuery, bool kSampled>
__global__ __launch_bounds__(kSpaThreads) void spa_split_hist_kernel(GView g, Emit E, SpaRound R) {
  R.n = uniform(round_items(R));
  __shared__ uint32_t lh[kSumBins];
  const uint32_t total = uniform(R.koff[R.n]);
  for (uint32_t q = blockIdx.x; q < total; q += gridDim.x) {
    const uint32_t j = uniform(spa_piece_source(R.koff, R.n, q));
    for (uint32_t b = threadIdx.x; b < kSumBins; b += kSpaThreads) lh[b] = 0;
    __syncthreads();
    const unsigned long long* HW = reinterpret_cast<const unsigned long long*>(R.acc + (uint64_t)j * g.n * 8);
    const uint32_t* K = R.keys + (uint64_t)j * g.n;
    const uint32_t nk = uniform(R.nkeys[j]);
    const uint32_t t = (q - uniform(R.koff[j])) * kSpaPiece + threadIdx.x;
    if (t < nk) {
      const unsigned long long v = HW[K[t]];
      if (v != 0) atomicAdd(&lh[sum_bin(v)], 1u);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kSumBins; b += kSpaThreads)
      if (lh[b]) atomicAdd(&R.hist[(uint64_t)j * kSumBins + b], lh[b]);
    __syncthreads();
  }
}

// one wave per source of the round
__global__ __launch_bounds__(64) void spa_split_floor_kernel(SpaRound R, uint32_t kq) {
  R.n = round_items(R);
  const uint32_t j = blockIdx.x;
  if (j >= R.n) return;
  const uint64_t f = sum_floor_wave(R.hist + (uint64_t)j * kSumBins, kq);
  if (lane_id() == 0) R.floor_sum[j] = f;
}

// score and emit pieces of 1024 keys, clearing the slab behind them
template <bool kW, bool kQuery, bool kSampled>
__global__ __launch_bounds__(kSpaThreads) void spa_split_sweep_kernel(GView g, Emit E, SpaRound R) {
  R.n = uniform(round_items(R));
  constexpr int NW = kSpaThreads / 64;
  __shared__ uint32_t st_c[NW][kSpaStage], st_h[NW][kSpaStage], st_k[NW][kSpaStage],
      st_d[NW][kSpaStage], st_w2[kW ? NW : 1][kW ? kSpaStage : 1];
  __shared__ uint32_t so_s[NW][64], so_a[NW][64], so_c[NW][64];
  const int wv = threadIdx.x >> 6;
  Stage SG{st_c[wv], st_h[wv], kW ? st_w2[wv] : nullptr, st_k[wv], st_d[wv], (uint32_t)kSpaStage,
           so_s[wv], so_a[wv], so_c[wv], 64u};
  FpAcc fa;
  WorkAcc wk;
  const uint32_t total = uniform(R.koff[R.n]);
  for (uint32_t q = blockIdx.x; q < total; q += gridDim.x) {
    const uint32_t j = uniform(spa_piece_source(R.koff, R.n, q));
    const SrcRec s = uniform_rec(load_rec(R.wl, R.i0 + j));
    const uint32_t ts_bits = E.fp_mode ? 0u : uniform((kQuery ? E.tau : tau_of(E, s.key))[0]);
    uint64_t wmin = kW ? min_wsum(E.measure, ts_bits, E.shift) : 1ull;
    if (kQuery && kW && R.floor_sum) {
      const uint64_t f = uniform64(R.floor_sum[j]);
      wmin = f > wmin ? f : wmin;
    }
    const uint32_t hmin = kW ? 1u : min_count(E.measure, ts_bits, s.da, !kQuery);
    char* slab = R.acc + (uint64_t)j * g.n * 8;
    const uint32_t* K = R.keys + (uint64_t)j * g.n;
    const uint32_t nk = uniform(R.nkeys[j]);
    const uint32_t t = (q - uniform(R.koff[j])) * kSpaPiece + threadIdx.x;
    uint32_t c = 0, h = 0;
    uint64_t wsum = 0;
    bool ok = false;
    if (t < nk) {
      // every key is listed once, and the accumulation is over (an earlier
      // launch): a plain read and clear, no read-modify-write atomics
      c = K[t];
      if (kW) {
        unsigned long long* p = reinterpret_cast<unsigned long long*>(slab) + c;
        wsum = *p;
        *p = 0ull;
        wk.v[4] += wsum != 0 ? 1u : 0u;
        ok = wsum != 0 && wsum >= wmin;
      } else {
        uint32_t* p = reinterpret_cast<uint32_t*>(slab) + c;
        h = *p;
        *p = 0u;
        wk.v[4] += h != 0 ? 1u : 0u;
        ok = h != 0 && h >= hmin;
      }
    }
    stage_add<kQuery, kW>(E, g, SG, ok, c, h, wsum, s.key, s.da, fa);
  }
  stage_drain<kQuery, kW>(E, g, SG, fa);
  flush_fp(E, fa);
  flush_work(E, wk);
}

// ---------------------------------------------------------------------------
// Radix select over the candidate buffer: the k largest keys
// (score bits, ~a, ~c), 9 digit steps of 11 / 11 / 10 bits per key word.
// ---------------------------------------------------------------------------

struct SelState {
  unsigned long long n_cur;  // entries in the working set
  unsigned long long k_rem;  // entries still to take from it
  unsigned long long n_out;  // entries emitted
  unsigned long long n_next;
  uint32_t digit;
  uint32_t take_all;  // the boundary bin is taken whole
  uint32_t done;
  uint32_t prefix[3];  // boundary key digits found so far (key words, bits above the step)
  uint32_t pad;
  // this step's reservations: entries emitted in the high half, entries of
  // the next working set in the low half (each < 2^32: n_cur < 2^32)
  unsigned long long step_pack;
};

__device__ inline void step_geom(int step, int* word, int* shift, int* bits) {
  *word = step / 3;
  const int r = step % 3;
  *shift = r == 0 ? 21 : (r == 1 ? 10 : 0);
  *bits = r == 2 ? 10 : 11;
}

__device__ inline uint32_t key_word(uint32_t s, uint32_t a, uint32_t c, int word) {
  return word == 0 ? s : (word == 1 ? ~a : ~c);
}

__global__ __launch_bounds__(256) void sel_hist_kernel(const uint32_t* __restrict__ ks,
                                                       const uint32_t* __restrict__ ka,
                                                       const uint32_t* __restrict__ kc,
                                                       const SelState* __restrict__ st, int step,
                                                       uint32_t* __restrict__ hist) {
  __shared__ uint32_t lh[2048];
  if (st->done) return;
  const unsigned long long n = st->n_cur;
  int word, shift, bits;
  step_geom(step, &word, &shift, &bits);
  const uint32_t mask = (1u << bits) - 1;
  for (int i = threadIdx.x; i < 2048; i += 256) lh[i] = 0;
  __syncthreads();
  for (unsigned long long i = (unsigned long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * 256) {
    const uint32_t kw = word == 0 ? ks[i] : (word == 1 ? ~ka[i] : ~kc[i]);
    atomicAdd(&lh[(kw >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2048; i += 256)
    if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

// Find the digit whose bin holds the k_rem-th largest key: 64 threads each
// sum 32 bins (from the top), a wave scan locates the thread, which then
// walks its own 32 bins.
__global__ __launch_bounds__(64) void sel_pick_kernel(SelState* st, int step, uint32_t* hist) {
  if (st->done) return;
  int word, shift, bits;
  step_geom(step, &word, &shift, &bits);
  const int nbins = 1 << bits;
  const int per = nbins / 64;
  const int t = threadIdx.x;
  const int top = nbins - 1 - t * per;  // this thread's bins: top, top - 1, ..., top - per + 1
  unsigned long long sum = 0;
  for (int j = 0; j < per; j++) sum += hist[top - j];
  unsigned long long incl = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(incl, o, 64);
    if (t >= o) incl += y;
  }
  const unsigned long long k = st->k_rem;
  const uint64_t hit = __ballot(incl >= k);
  const int owner = hit ? __ffsll((unsigned long long)hit) - 1 : 63;
  if (t == owner) {
    unsigned long long above = incl - sum;
    int d = top;
    for (int j = 0; j < per; j++, d--) {
      if (above + hist[d] >= k) break;
      above += hist[d];
    }
    if (d < top - per + 1) d = top - per + 1;
    st->digit = (uint32_t)d;
    st->take_all = (above + hist[d] == k) ? 1u : 0u;
    st->k_rem = k - above;
    st->prefix[word] |= ((uint32_t)d) << shift;
    st->n_next = 0;
    st->step_pack = 0;
  }
  __syncthreads();
  for (int i = t; i < 2048; i += 64) hist[i] = 0;
}

constexpr int kSelItems = 16;  // elements per thread per tile of the partition

// Partition the working set around the chosen digit: larger digits go to the
// output, the boundary digit to the next working set.  Each block owns a
// contiguous chunk of tiles of 256 * kSelItems entries: it counts both
// classes over the chunk (key word only), reserves its two ranges with one
// 64-bit atomic on step_pack, then classifies again and writes the chunk tile
// by tile.  Same-address atomics serialise, so there is one per block, not
// one per tile.
__global__ __launch_bounds__(256) void sel_partition_kernel(
    const uint32_t* __restrict__ ks, const uint32_t* __restrict__ ka, const uint32_t* __restrict__ kc,
    SelState* st, int step, uint32_t* __restrict__ ns, uint32_t* __restrict__ na,
    uint32_t* __restrict__ nc, uint32_t* __restrict__ os, uint32_t* __restrict__ oa,
    uint32_t* __restrict__ oc) {
  __shared__ uint32_t w_out[4], w_next[4];
  __shared__ unsigned long long b_out, b_next;
  if (st->done) return;
  const unsigned long long n = st->n_cur;
  int word, shift, bits;
  step_geom(step, &word, &shift, &bits);
  const uint32_t mask = (1u << bits) - 1;
  const uint32_t dsel = st->digit;
  const bool take_all = st->take_all != 0;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  constexpr unsigned long long kTile = 256ull * kSelItems;
  const unsigned long long ntiles = (n + kTile - 1) / kTile;
  const unsigned long long per = (ntiles + gridDim.x - 1) / gridDim.x;
  const unsigned long long c_begin = (unsigned long long)blockIdx.x * per * kTile;
  const unsigned long long c_end = c_begin + per * kTile < n ? c_begin + per * kTile : n;
  if (c_begin >= c_end) return;  // uniform over the block
  const uint32_t* kp = word == 0 ? ks : (word == 1 ? ka : kc);
  const uint32_t kinv = word == 0 ? 0u : ~0u;  // key words 1 and 2 are ~a and ~c
  // pass 1: the chunk's class counts
  uint32_t n_o = 0, n_n = 0;
  for (unsigned long long i = c_begin + threadIdx.x; i < c_end; i += 256) {
    const uint32_t d = ((kp[i] ^ kinv) >> shift) & mask;
    n_o += (d > dsel || (take_all && d == dsel)) ? 1u : 0u;
    n_n += (!take_all && d == dsel) ? 1u : 0u;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    n_o += __shfl_xor(n_o, o);
    n_n += __shfl_xor(n_n, o);
  }
  if (lane == 0) {
    w_out[wid] = n_o;
    w_next[wid] = n_n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long to = (unsigned long long)w_out[0] + w_out[1] + w_out[2] + w_out[3];
    const unsigned long long tn = (unsigned long long)w_next[0] + w_next[1] + w_next[2] + w_next[3];
    const unsigned long long old = (to | tn) ? atomicAdd(&st->step_pack, (to << 32) | tn) : 0ull;
    b_out = st->n_out + (old >> 32);
    b_next = old & 0xFFFFFFFFull;
  }
  __syncthreads();
  unsigned long long run_out = b_out, run_next = b_next;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // pass 2: classify and write, tile by tile.  Entries are ranked in (wave,
  // item, lane) order, so the lanes of one store write a contiguous run.
  for (unsigned long long t0 = c_begin; t0 < c_end; t0 += kTile) {
    uint32_t cls = 0;  // 2 bits per item: 1 = out, 2 = next
    uint32_t c_out = 0, c_next = 0;  // this wave's totals (uniform)
#pragma unroll
    for (int j = 0; j < kSelItems; j++) {
      const unsigned long long i = t0 + (unsigned long long)j * 256 + threadIdx.x;
      uint32_t cl = 0;
      if (i < c_end) {
        const uint32_t d = ((kp[i] ^ kinv) >> shift) & mask;
        cl = (d > dsel || (take_all && d == dsel)) ? 1u : (d == dsel ? 2u : 0u);
      }
      cls |= cl << (2 * j);
      c_out += (uint32_t)__popcll(__ballot(cl == 1u));
      c_next += (uint32_t)__popcll(__ballot(cl == 2u));
    }
    if (lane == 0) {
      w_out[wid] = c_out;
      w_next[wid] = c_next;
    }
    __syncthreads();
    unsigned long long po = run_out, pn = run_next;
    for (int w = 0; w < 4; w++) {
      if (w < wid) {
        po += w_out[w];
        pn += w_next[w];
      }
      run_out += w_out[w];
      run_next += w_next[w];
    }
#pragma unroll
    for (int j = 0; j < kSelItems; j++) {
      const uint32_t cl = (cls >> (2 * j)) & 3u;
      const uint64_t bo = __ballot(cl == 1u), bn = __ballot(cl == 2u);
      const unsigned long long i = t0 + (unsigned long long)j * 256 + threadIdx.x;
      if (cl == 1u) {
        const unsigned long long q = po + (unsigned long long)__popcll(bo & lt);
        os[q] = ks[i];
        oa[q] = ka[i];
        oc[q] = kc[i];
      } else if (cl == 2u) {
        const unsigned long long q = pn + (unsigned long long)__popcll(bn & lt);
        ns[q] = ks[i];
        na[q] = ka[i];
        nc[q] = kc[i];
      }
      po += (unsigned long long)__popcll(bo);
      pn += (unsigned long long)__popcll(bn);
    }
    __syncthreads();
  }
}

__global__ void sel_advance_kernel(SelState* st, int last_step) {
  if (st->done) return;
  st->n_out += st->step_pack >> 32;
  st->n_next = st->step_pack & 0xFFFFFFFFull;
  if (st->take_all || last_step) {
    st->done = 1;
    return;
  }
  st->n_cur = st->n_next;
}

__global__ void sel_init_kernel(SelState* st, const unsigned long long* count,
                                unsigned long long cap, unsigned long long base,
                                unsigned long long k) {
  unsigned long long n = *count;
  if (n > cap) n = cap;
  n = n > base ? n - base : 0;
  st->n_cur = n;
  st->n_out = 0;
  st->n_next = 0;
  st->prefix[0] = st->prefix[1] = st->prefix[2] = 0;
  st->take_all = 0;
  st->digit = 0;
  st->k_rem = k < n ? k : n;
  st->done = (k >= n) ? 2u : 0u;  // 2: everything is selected (copied separately)
}

__global__ void sel_copy_all_kernel(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ ka,
                                    const uint32_t* __restrict__ kc, SelState* st,
                                    uint32_t* __restrict__ os, uint32_t* __restrict__ oa,
                                    uint32_t* __restrict__ oc) {
  if (st->done != 2) return;
  const unsigned long long n = st->n_cur;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    os[i] = ks[i];
    oa[i] = ka[i];
    oc[i] = kc[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st->n_out = n;
}

// tau from the boundary prefix: the k-th largest key is >= prefix (remaining bits 0)
__global__ void sel_tau_kernel(const SelState* st, uint32_t* tau) {
  if (st->done == 2 || st->n_cur == 0) {
    tau[0] = tau[1] = tau[2] = 0;
    return;
  }
  tau[0] = st->prefix[0];
  tau[1] = st->prefix[1];
  tau[2] = st->prefix[2];
}

__global__ void write_out_kernel(const uint32_t* __restrict__ s, const uint32_t* __restrict__ a,
                                 const uint32_t* __restrict__ c, unsigned long long k,
                                 int32_t* __restrict__ oa, int32_t* __restrict__ oc,
                                 float* __restrict__ os) {
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < k;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    oa[i] = (int32_t)a[i];
    oc[i] = (int32_t)c[i];
    os[i] = __uint_as_float(s[i]);
  }
}

// ---------------------------------------------------------------------------
// Query result: per query index, the first k_q entries of its sorted segment
// ---------------------------------------------------------------------------

__global__ void query_take_kernel(const uint32_t* __restrict__ s, const uint32_t* __restrict__ c,
                                  const uint32_t* __restrict__ seg_start,
                                  const uint32_t* __restrict__ seg_count, uint32_t nq, int32_t kq,
                                  int32_t* __restrict__ out_c, float* __restrict__ out_s,
                                  int32_t* __restrict__ out_count, const uint32_t* __restrict__ nq_dev,
                                  uint64_t cap) {
  // nq_dev: the query count is read on the device (at most nq); cap: the
  // candidate buffer's size (a call whose candidates outgrew it is discarded
  // by the host, but its reads stay inside the buffer)
  if (nq_dev) nq = min(*nq_dev, nq);
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < (uint64_t)nq * kq;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t q = (uint32_t)(t / (uint32_t)kq), j = (uint32_t)(t % (uint32_t)kq);
    const uint32_t m = seg_count[q] < (uint32_t)kq ? seg_count[q] : (uint32_t)kq;
    if (j == 0) out_count[q] = (int32_t)m;
    if (j < m && (uint64_t)seg_start[q] + j < cap) {
      out_c[t] = (int32_t)c[seg_start[q] + j];
      out_s[t] = __uint_as_float(s[seg_start[q] + j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------

static GView view_of(const lp_graph* g) {
  GView v;
  v.off = g->off;
  v.adj = g->adj;
  v.hoff = g->hoff;
  v.hdeg = g->hdeg;
  v.hstart = g->hstart;
  v.hpsum = g->hpsum;
  v.deg = g->deg;
  v.below = g->below;
  v.perm = g->perm;
  v.deg_first = g->deg_first;
  v.deg_cap = g->deg_cap;
  v.n = (uint32_t)g->n;
  return v;
}

static unsigned grid_for(uint64_t items, int per_block, unsigned cap_blocks) {
  uint64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap_blocks) b = cap_blocks;
  return (unsigned)b;
}

// Wedge budget of the sampling pass: the tuning's, else about 0.1% of the
// wedges, clamped to [2^20, 2^22] (the sample's launches are latency bound,
// so a larger one costs time and a smaller one loosens the threshold); 0
// turns sampling off.
static uint64_t sample_budget(const lp_graph* g, uint64_t total_w) {
  if (g->tuning.sample_budget < 0) return 0;
  if (g->tuning.sample_budget > 0) return (uint64_t)g->tuning.sample_budget;
  return std::min<uint64_t>(1ull << 22, std::max<uint64_t>(1ull << 20, total_w >> 10));
}

struct AccConfig {
  BucketCuts cuts;    // bucket bounds; cuts.t[kBucketLarge]: T above which a source uses the global path
  unsigned spa_wgs;   // workgroups (dense accumulators) of the global path
};

static AccConfig acc_config(const lp_graph* g) {
  AccConfig c;
  for (int b = kBucketTiny; b < kBucketLarge; b++)
    c.cuts.t[b] = (uint32_t)(g->tuning.bucket_max[b] > 0 ? g->tuning.bucket_max[b] : kBucketMaxDefault[b]);
  c.cuts.t[kBucketLarge] = g->tuning.lds_wedge_cap > 0
                               ? (uint32_t)std::min<int64_t>(g->tuning.lds_wedge_cap, 1u << 30)
                               : 65536u;
  c.spa_wgs = (unsigned)(g->tuning.global_slots > 0 ? g->tuning.global_slots : num_cus());
  return c;
}

template <int TM, bool kQuery, bool kSampled>
static lp_status launch_bucket_tables(lp_graph* g, int bucket, const GView& gv, const Emit& E,
                                      WorkList wl, uint64_t nitems, hipStream_t st);

// Kernel shapes a tuning may pick for the small and mid1 buckets
// (lp_tuning.kernel_shape; 0 keeps the default).
enum : int {
  kShapeBatch = 1,          // several sources share a workgroup and one table
  kShapeWave = 2,           // one source per 64-lane wave, four per workgroup (small only)
  kShapeWorkgroup128 = 3,   // one source per 128-lane workgroup
  kShapeWorkgroup256 = 4    // one source per 256-lane workgroup
};

// Launch the accumulation of one work list in the given bucket.
template <int TM, bool kQuery, bool kSampled>
static lp_status launch_bucket(lp_graph* g, int bucket, const GView& gv, const Emit& E,
                               WorkList wl, uint64_t nitems, hipStream_t st) {
  if (nitems == 0) return LP_OK;
  const unsigned cus = (unsigned)num_cus();
  // kernel shapes of the small and mid1 buckets (prediction orientation):
  // batches of sources sharing a workgroup and a table, or one source per
  // wave / per 128 / 256 lanes; the default depends on the table kind
  if (!kQuery && (bucket == kBucketSmall || bucket == kBucketMid1)) {
    const int64_t shape = g->tuning.kernel_shape[bucket == kBucketSmall ? 0 : 1];
    // default: batches (fastest on R-MAT-22 with count tables and, taken
    // over AA at L = 32 and RA at L = 256, on Chung-Lu 8M with packed ones)
    const int sh = shape != 0 ? (int)shape : kShapeBatch;
    bool done = true;
    if (sh == kShapeWave)
      hipLaunchKernelGGL((acc_lds_kernel<256, 64, 384, TM, false, 128, kSampled>),
                         dim3(grid_for(nitems, 4, cus * 16)), dim3(256), 0, st, gv, E, wl);
    else if (sh == kShapeWorkgroup128)
      hipLaunchKernelGGL((acc_lds_kernel<128, 128, 1536, TM, false, 128, kSampled>),
                         dim3(grid_for(nitems, 1, cus * 16)), dim3(128), 0, st, gv, E, wl);
    else if (sh == kShapeWorkgroup256)
      hipLaunchKernelGGL((acc_lds_kernel<256, 256, TM == kTabPacked ? 3008 : 3072, TM, false, 64, kSampled>),
                         dim3(grid_for(nitems, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
    else
      done = false;
    if (done) {
      LP_HIP(hipGetLastError());
      return LP_OK;
    }
  }
  if constexpr (TM == kTabPacked) {
    // packed AA / RA tables (prediction orientation; keys hold the batch
    // position right above id_bits(n + 1) <= 25 bits).  Table sizes keep the
    // workgroups per CU of the count kernels (the packed kernels also hold the
    // 64-bit weight of each arc, retry entry and staged sum).
    switch (bucket) {
      case kBucketTiny:
        hipLaunchKernelGGL((acc_batch_kernel<256, 48, 2432, TM, 64, kSampled>),
                           dim3(grid_for((nitems + 47) / 48, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
        break;
      case kBucketSmall:
        hipLaunchKernelGGL((acc_batch_kernel<256, 8, 2816, TM, 64, kSampled>),
                           dim3(grid_for((nitems + 7) / 8, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
        break;
      case kBucketMid1:
        hipLaunchKernelGGL((acc_batch_kernel<512, 4, 5760, TM, 64, kSampled>),
                           dim3(grid_for((nitems + 3) / 4, 1, cus * 4)), dim3(512), 0, st, gv, E, wl);
        break;
      case kBucketMid2:
        hipLaunchKernelGGL((acc_lds_kernel<256, 256, 3008, TM, false, 64, kSampled>),
                           dim3(grid_for(nitems, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
        break;
      case kBucketMid3:
        hipLaunchKernelGGL((acc_lds_kernel<512, 512, 6016, TM, false, 64, kSampled>),
                           dim3(grid_for(nitems, 1, cus * 4)), dim3(512), 0, st, gv, E, wl);
        break;
      case kBucketLarge:
        hipLaunchKernelGGL((acc_lds_kernel<1024, 1024, 12032, TM, false, 64, kSampled>),
                           dim3(grid_for(nitems, 1, cus * 2)), dim3(1024), 0, st, gv, E, wl);
        break;
      default:
        return set_error(LP_ERR_INVALID_ARGUMENT, "bad bucket");
    }
    LP_HIP(hipGetLastError());
    return LP_OK;
  } else {
    return launch_bucket_tables<TM, kQuery, kSampled>(g, bucket, gv, E, wl, nitems, st);
  }
}

// Count tables and 12-byte weighted tables.
template <int TM, bool kQuery, bool kSampled>
static lp_status launch_bucket_tables(lp_graph* g, int bucket, const GView& gv, const Emit& E,
                                      WorkList wl, uint64_t nitems, hipStream_t st) {
  constexpr bool kW = TM != kTabCount;
  const unsigned cus = (unsigned)num_cus();
  const uint64_t n = (uint64_t)g->n;
  if (!kQuery && bucket <= kBucketMid1) {
    // batches: Tiny 48 sources (<= 1536 wedges; 32 above 2^26 vertices),
    // Small 8 (<= 2048), Mid1 4 per 512 lanes for count tables (<= 4096), 2
    // per 256 lanes for weighted ones (<= 2048)
    // (the tuning may ask for 32 tiny or 4 small sources per workgroup)
    const bool tiny32 = g->tuning.batch_sources[0] == 32;
    const bool small4 = g->tuning.batch_sources[1] == 4;
    bool done = true;
    if (bucket == kBucketTiny && !tiny32 && n <= BatchKey<48>::kMaxN)
      hipLaunchKernelGGL((acc_batch_kernel<256, 48, 3072, TM, 64, kSampled>),
                         dim3(grid_for((nitems + 47) / 48, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
    else if (bucket == kBucketTiny && n <= BatchKey<32>::kMaxN)
      hipLaunchKernelGGL((acc_batch_kernel<256, 32, 3072, TM, 64, kSampled>),
                         dim3(grid_for((nitems + 31) / 32, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
    else if (bucket == kBucketSmall && !small4 && n <= BatchKey<8>::kMaxN)
      hipLaunchKernelGGL((acc_batch_kernel<256, 8, 3072, TM, 64, kSampled>),
                         dim3(grid_for((nitems + 7) / 8, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
    else if (bucket == kBucketSmall && n <= BatchKey<4>::kMaxN)
      hipLaunchKernelGGL((acc_batch_kernel<256, 4, 3072, TM, 64, kSampled>),
                         dim3(grid_for((nitems + 3) / 4, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
    else if (bucket == kBucketMid1 && !kW && n <= BatchKey<4>::kMaxN)
      hipLaunchKernelGGL((acc_batch_kernel<512, 4, 6144, TM, 64, kSampled>),
                         dim3(grid_for((nitems + 3) / 4, 1, cus * 4)), dim3(512), 0, st, gv, E, wl);
    else if (bucket == kBucketMid1 && n <= BatchKey<2>::kMaxN)
      hipLaunchKernelGGL((acc_batch_kernel<256, 2, 3072, TM, 64, kSampled>),
                         dim3(grid_for((nitems + 1) / 2, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
    else
      done = false;
    if (done) {
      LP_HIP(hipGetLastError());
      return LP_OK;
    }
  }
  switch (bucket) {
    case kBucketTiny:
      hipLaunchKernelGGL((acc_lds_kernel<256, 64, 48, TM, kQuery, 128, kSampled>),
                         dim3(grid_for(nitems, 4, cus * 16)), dim3(256), 0, st, gv, E, wl);
      break;
    case kBucketSmall:
      hipLaunchKernelGGL((acc_lds_kernel<256, 64, 384, TM, kQuery, 128, kSampled>),
                         dim3(grid_for(nitems, 4, cus * 16)), dim3(256), 0, st, gv, E, wl);
      break;
    case kBucketMid1:
      hipLaunchKernelGGL((acc_lds_kernel<128, 128, 1536, TM, kQuery, 128, kSampled>),
                         dim3(grid_for(nitems, 1, cus * 16)), dim3(128), 0, st, gv, E, wl);
      break;
    case kBucketMid2:
      hipLaunchKernelGGL((acc_lds_kernel<256, 256, 3072, TM, kQuery, 64, kSampled>),
                         dim3(grid_for(nitems, 1, cus * 8)), dim3(256), 0, st, gv, E, wl);
      break;
    case kBucketMid3:
      hipLaunchKernelGGL((acc_lds_kernel<512, 512, kW ? 4608 : 6144, TM, kQuery, 64, kSampled>),
                         dim3(grid_for(nitems, 1, cus * 4)), dim3(512), 0, st, gv, E, wl);
      break;
    case kBucketLarge:
      hipLaunchKernelGGL((acc_lds_kernel<1024, 1024, kW ? 7680 : 14336, TM, kQuery, 64, kSampled>),
                         dim3(grid_for(nitems, 1, cus * 2)), dim3(1024), 0, st, gv, E, wl);
      break;
    default:
      return set_error(LP_ERR_INVALID_ARGUMENT, "bad bucket");
  }
  LP_HIP(hipGetLastError());
  return LP_OK;
}

template <bool kW, bool kQuery, bool kSampled>
static lp_status launch_spa(lp_graph* g, Workspace& w, const GView& gv, const Emit& E, WorkList wl,
                            SpaItem ov, uint64_t nitems, hipStream_t st) {
  if (nitems == 0) return LP_OK;
  AccConfig cfg = acc_config(g);
  const size_t n = (size_t)g->n;
  // pool: one slab of 8n accumulator bytes per workgroup, then as many key
  // lists of 4n; it grows to the launch's workgroup count (at most
  // cfg.spa_wgs, and at most an eighth of the device memory, since every
  // server slot has a workspace of its own) and never shrinks
  uint64_t mem_cap = std::max<uint64_t>(1, device_memory() / 8 / (n * 12 + 1));
  if (w.global_tab.fixed) {
    // a workspace over fixed memory holds as many slabs as fit
    mem_cap = w.global_tab.cap / (n * 12);
    if (mem_cap == 0)
      return set_error(LP_ERR_INVALID_ARGUMENT,
                       "a source above the LDS capacity needs a dense accumulator of %zu bytes; the fixed "
                       "scratch holds %zu",
                       n * 12, w.global_tab.cap);
  }
  const unsigned slabs = (unsigned)std::min<uint64_t>(std::min<uint64_t>(cfg.spa_wgs, nitems), mem_cap);
  if (w.global_slabs < slabs) {
    w.global_tab.release();
    w.global_slabs = 0;
    LP_TRY(w.global_tab.ensure((size_t)slabs * n * 12));
    LP_HIP(hipMemsetAsync(w.global_tab.p, 0, (size_t)slabs * n * 8, st));
    w.global_slabs = slabs;
  }
  // the accumulators are left zeroed by every workgroup; the key lists need no init
  char* base = w.global_tab.as<char>();
  uint32_t* spa_keys = reinterpret_cast<uint32_t*>(base + (size_t)w.global_slabs * n * 8);
  if (ov.ovf || nitems > 2ull * slabs) {
    // one workgroup per source (or overflow record), its own slab: with many
    // sources (more than two rounds of slabs) every CU has one and no round
    // waits for its slowest piece.  Overflow records (partitions of sources
    // that filled an LDS table) always go here.
    hipLaunchKernelGGL((acc_spa_kernel<kW, kQuery, kSampled>), dim3(slabs), dim3(kSpaThreads), 0, st, gv, E,
                       wl, ov, base, spa_keys);
    LP_HIP(hipGetLastError());
    return LP_OK;
  }
  // few sources (at most two rounds): one workgroup each would leave the GPU
  // idle behind the largest, so each is split over all CUs
  // meta: poff, koff, nkeys (u32, slabs + 1 each), then per-source floors
  // (u64) and sum histograms (u32, kSumBins each)
  const size_t u32_meta = ((size_t)slabs * 3 + 8 + 1) & ~(size_t)1;
  const bool floors = kQuery && kW && E.kq > 0;
  LP_TRY(w.spa_meta.ensure(u32_meta * 4 + (size_t)slabs * 8 + (floors ? (size_t)slabs * kSumBins * 4 : 0)));
  uint32_t* meta = w.spa_meta.as<uint32_t>();
  unsigned long long* floor_sum = reinterpret_cast<unsigned long long*>(meta + u32_meta);
  uint32_t* hist = reinterpret_cast<uint32_t*>(floor_sum + slabs);
  const unsigned grid = (unsigned)num_cus() * 4;
  for (uint64_t r0 = 0; r0 < nitems; r0 += slabs) {
    const uint32_t nr = (uint32_t)std::min<uint64_t>(slabs, nitems - r0);
    SpaRound R{wl,   (uint32_t)r0, nr,   meta, meta + slabs + 1, meta + 2 * (slabs + 1), base, spa_keys,
               hist, floors ? floor_sum : nullptr};
    LP_HIP(hipMemsetAsync(R.nkeys, 0, (size_t)nr * 4, st));
    hipLaunchKernelGGL(spa_pieces_kernel, dim3(1), dim3(1024), 0, st, R, 0);
    hipLaunchKernelGGL((spa_split_acc_kernel<kW, kQuery, kSampled>), dim3(grid), dim3(kSpaThreads), 0, st, gv,
                       E, R);
    hipLaunchKernelGGL((spa_split_excl_kernel<kW, kQuery, kSampled>), dim3(nr), dim3(kSpaThreads), 0, st, gv, E,
                       R);
    hipLaunchKernelGGL(spa_pieces_kernel, dim3(1), dim3(1024), 0, st, R, 1);
    if (floors) {
      LP_HIP(hipMemsetAsync(hist, 0, (size_t)nr * kSumBins * 4, st));
      hipLaunchKernelGGL((spa_split_hist_kernel<kW, kQuery, kSampled>), dim3(grid), dim3(kSpaThreads), 0, st,
                         gv, E, R);
      hipLaunchKernelGGL(spa_split_floor_kernel, dim3(nr), dim3(64), 0, st, R, E.kq);
    }
    hipLaunchKernelGGL((spa_split_sweep_kernel<kW, kQuery, kSampled>), dim3(grid), dim3(kSpaThreads), 0, st, gv,
                       E, R);
    LP_HIP(hipGetLastError());
  }
  return LP_OK;
}

// HIP events around every accumulation launch of a call, on the call's
// stream; per-bucket device time and launch counts go to the call's stats.
// The events belong to the workspace (created on its first call), so a call
// records them and creates none.
static hipEvent_t* workspace_events(hipEvent_t* ev, int n) {
  for (int i = 0; i < n; i++)
    if (!ev[i]) (void)hipEventCreate(&ev[i]);
  return ev;
}

struct LaunchClock {
  static_assert(kBuckets == kNumBuckets, "one clock slot pair per bucket");
  // per pass (main, then sampling), kBuckets + 2 slots: the buckets, the
  // global-path launch for overflowing LDS tables (counted as global), and
  // the 12-byte-table launch for sources whose packed sums do not fit (split)
  static constexpr int kSlots = kBuckets + 2;
  hipEvent_t* ev;
  bool used[2 * kSlots] = {};
  lp_stats* stats = nullptr;
  LaunchClock(lp_stats* s, Workspace& w) : ev(workspace_events(w.clock_ev, 4 * kSlots)), stats(s) {}
  lp_status start(int slot, hipStream_t st) {
    used[slot] = true;
    LP_HIP(hipEventRecord(ev[2 * slot], st));
    return LP_OK;
  }
  lp_status stop(int slot, hipStream_t st) {
    LP_HIP(hipEventRecord(ev[2 * slot + 1], st));
    return LP_OK;
  }
  // after the stream has passed every stop event
  void collect() {
    for (int s = 0; s < 2 * kSlots; s++) {
      if (!used[s]) continue;
      float t = 0;
      if (hipEventElapsedTime(&t, ev[2 * s], ev[2 * s + 1]) != hipSuccess) (void)hipGetLastError();
      const int r = s % kSlots;
      lp_bucket_stats* arr = s >= kSlots ? stats->sampled : stats->bucket;
      lp_bucket_stats& b = arr[r < kBuckets ? r : (r == kBuckets ? kBucketHuge : kStatRows - 1)];
      b.ms += t;
      b.launches += 1;
      used[s] = false;
    }
  }
};

// Work counters of the launches of one call: 8 uint64 per bucket, main pass
// first, then the sampling pass.
static unsigned long long* work_counters(Workspace& w) {
  return reinterpret_cast<unsigned long long*>(w.counters.as<char>() + 1024);
}
constexpr int kSampledWork = 8 * 8;  // offset of the sampling pass's counters

static void fill_work(const unsigned long long* h, lp_stats* S) {
  for (int p = 0; p < 2; p++) {
    lp_bucket_stats* arr = p ? S->sampled : S->bucket;
    const unsigned long long* x = h + p * kSampledWork;
    for (int b = 0; b < kStatRows; b++) {
      arr[b].sources = x[b * 8 + 0];
      arr[b].first_order = x[b * 8 + 1];
      arr[b].arcs = x[b * 8 + 2];
      arr[b].wedges = x[b * 8 + 3];
      arr[b].candidates = x[b * 8 + 4];
    }
  }
}

// Device values the caller reads after a phase, fetched in the phase's own
// host round trip (after any overflow launch).
// Small device -> host reads of one host round trip.  A copy into pageable
// memory blocks the host by itself, so the values land in the workspace's
// pinned buffer (after the plan summary) and reach the caller's variables
// when finish() has synchronised the stream.
constexpr size_t kHostStatsBytes = 4096;
constexpr size_t kStageBase = 256;  // the plan summary sits below
static_assert(sizeof(PlanOut) <= kStageBase, "plan summary overlaps the readback staging");

struct PinnedReads {
  static constexpr int kMax = 8;
  Workspace& w;
  int n = 0;
  size_t used = 0;
  void* dst[kMax];
  size_t off[kMax], bytes[kMax];
  explicit PinnedReads(Workspace& ws) : w(ws) {}
  lp_status add(void* d, const void* src, size_t b, hipStream_t st) {
    LP_TRY(w.host_stats.ensure(kHostStatsBytes));
    if (n == kMax || kStageBase + used + b > kHostStatsBytes)
      return set_error(LP_ERR_DEVICE, "readback staging full");
    LP_HIP(hipMemcpyAsync(w.host_stats.as<char>() + kStageBase + used, src, b,
                          hipMemcpyDeviceToHost, st));
    dst[n] = d;
    off[n] = kStageBase + used;
    bytes[n] = b;
    n++;
    used = (used + b + 15) & ~(size_t)15;
    return LP_OK;
  }
  lp_status finish(hipStream_t st) {
    LP_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n; i++) std::memcpy(dst[i], w.host_stats.as<char>() + off[i], bytes[i]);
    n = 0;
    used = 0;
    return LP_OK;
  }
};

struct Readback {
  void* dst[2] = {nullptr, nullptr};
  const void* src[2] = {nullptr, nullptr};
  size_t bytes[2] = {0, 0};
  lp_status issue(PinnedReads& pr, hipStream_t st) const {
    for (int i = 0; i < 2; i++)
      if (bytes[i]) LP_TRY(pr.add(dst[i], src[i], bytes[i], st));
    return LP_OK;
  }
};

static lp_status collect_work(Workspace& w, lp_stats* S, hipStream_t st) {
  unsigned long long h[2 * kSampledWork];
  PinnedReads reads(w);
  LP_TRY(reads.add(h, work_counters(w), sizeof(h), st));
  LP_TRY(reads.finish(st));
  fill_work(h, S);
  return LP_OK;
}

// The whole accumulation for one phase (all buckets, then overflow records).
// ---------------------------------------------------------------------------
// AA / RA with a threshold (Section 3.1 sums): every sum a source accumulates
// adds the fixed-point weights of a subset of its explored arcs, so a source
// whose arcs' weights together stay below the threshold sum has no key that
// can pass.  This kernel copies the other records of a work list to out (in
// any order; their count lands in *out_count), so that the accumulation
// launch skips the rest whole.  A workgroup takes tiles of kPruneTile
// records, each wave groups of 64: their arcs are walked as one flat range,
// kWin windows of 64 at a time, each arc's weight added to its record's sum
// in LDS.  The survivors of a tile take their output slots with one atomic.
// ---------------------------------------------------------------------------
constexpr int kPruneGroups = 4;                        // groups of 64 records per wave and tile
constexpr uint32_t kPruneTile = 4 * 64 * kPruneGroups;  // records per workgroup and tile

__global__ __launch_bounds__(256) void prune_weighted_kernel(GView g, Emit E, WorkList wl,
                                                             SrcRec* __restrict__ out,
                                                             uint32_t* __restrict__ out_count) {
  __shared__ uint32_t s_excl[4][64];
  __shared__ uint32_t s_h0[4][64];
  __shared__ unsigned long long s_sum[4][64];
  __shared__ uint8_t s_mark[4][64];
  __shared__ uint32_t s_kept[4];
  __shared__ uint32_t s_at;
  const int wv = threadIdx.x >> 6;
  const uint32_t lane = (uint32_t)lane_id();
  uint32_t* excl = s_excl[wv];
  uint32_t* h0 = s_h0[wv];
  unsigned long long* sum = s_sum[wv];
  uint8_t* mark = s_mark[wv];
  mark[lane] = 0;
  const uint32_t total = uniform(work_count(wl));
  for (uint32_t tile = blockIdx.x * kPruneTile; tile < total; tile += gridDim.x * kPruneTile) {
    SrcRec rec[kPruneGroups];
    uint64_t M[kPruneGroups];
    uint32_t nkept = 0;
#pragma unroll
    for (int q = 0; q < kPruneGroups; q++) {
      const uint32_t base = tile + (uint32_t)(wv * kPruneGroups + q) * 64u;
      const uint32_t i = base + lane;
      const bool in = i < total;
      SrcRec r{};
      if (in) r = load_rec(wl, i);
      const uint32_t nrec = base < total ? uniform(total - base < 64u ? total - base : 64u) : 0u;
      // a listed source has wedges, so it explores at least one arc: the
      // records' arc ranges are never empty, as the window decoder needs
      uint32_t x = r.na;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
      }
      const uint32_t NA = uniform(__shfl(x, 63, 64));
      excl[lane] = x - r.na;
      h0[lane] = r.h0;
      sum[lane] = 0;
      wave_fence();
      uint32_t j = 0;
      for (uint32_t f = 0; f < NA; f += 64 * kWin) {
        uint32_t d[kWin], ri[kWin];
        bool v[kWin];
#pragma unroll
        for (int u = 0; u < kWin; u++) {
          const uint32_t fb = f + 64u * u;
          ri[u] = 0;
          v[u] = false;
          uint32_t e = 0;
          if (fb < NA) {
            ri[u] = decode_window(excl, nrec, mark, fb, j);
            v[u] = fb + lane < NA;
            if (v[u]) e = h0[ri[u]] + (fb + lane - excl[ri[u]]);
          }
          d[u] = g.hdeg[e];
        }
#pragma unroll
        for (int u = 0; u < kWin; u++)
          if (v[u]) atomicAdd(&sum[ri[u]], (unsigned long long)weight_of(E.measure, d[u], E.shift));
      }
      wave_fence();
      const bool keep = in && sum[lane] >= min_wsum(E.measure, tau_of(E, r.key)[0], E.shift);
      wave_fence();  // the sums are read before the next group resets them
      rec[q] = r;
      M[q] = __ballot(keep);
      nkept += (uint32_t)__popcll(M[q]);
    }
    if (lane == 0) s_kept[wv] = nkept;
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t t = s_kept[0] + s_kept[1] + s_kept[2] + s_kept[3];
      s_at = t ? atomicAdd(out_count, t) : 0u;
    }
    __syncthreads();
    uint32_t at = s_at;
    for (int w = 0; w < wv; w++) at += s_kept[w];
    at = uniform(at);
#pragma unroll
    for (int q = 0; q < kPruneGroups; q++) {
      if ((M[q] >> lane) & 1) out[at + rank_lt(M[q])] = rec[q];
      at += (uint32_t)__popcll(M[q]);
    }
    __syncthreads();  // s_kept and s_at are read before the next tile writes them
  }
}

template <int TM, bool kQuery>
static lp_status run_phase(lp_graph* g, Workspace& w, const GView& gv, const Emit& E0,
                           const SrcRec* lists, uint64_t list_stride, const uint32_t* counts_host,
                           uint32_t stride, int phase, uint32_t* ovf_host_count, LaunchClock* clk,
                           hipStream_t st, const uint32_t* first = nullptr,
                           const Readback* rb = nullptr, bool prune = false) {
  constexpr bool kW = TM != kTabCount;
  unsigned long long* work = work_counters(w);
  auto items_of = [&](int b) -> uint64_t {
    if (phase == 0 || stride <= 1) return phase == 2 ? 0 : counts_host[b];
    const uint64_t ns = (counts_host[b] + stride - 1) / stride;
    return phase == 1 ? ns : counts_host[b] - ns;
  };
  // AA / RA with a threshold: the batched buckets (tiny, small, mid1) first
  // drop the sources whose arcs' weights cannot reach it; the survivors go to
  // per-bucket lists whose lengths the accumulation kernels read on the device
  SrcRec* kept = nullptr;
  uint32_t* kept_count = nullptr;
  uint64_t kept_off[kBucketMid1 + 2] = {};
  if (kW && !kQuery && prune && phase != 1) {
    for (int b = 0; b <= kBucketMid1; b++) kept_off[b + 1] = kept_off[b] + items_of(b);
    if (kept_off[kBucketMid1 + 1] > 0) {
      LP_TRY(w.kept.ensure(256 + kept_off[kBucketMid1 + 1] * sizeof(SrcRec)));
      kept_count = w.kept.as<uint32_t>();
      kept = reinterpret_cast<SrcRec*>(w.kept.as<char>() + 256);
      LP_HIP(hipMemsetAsync(kept_count, 0, 4 * (kBucketMid1 + 1), st));
    }
  }
  // The sampling phase launches every bucket with a few sources each: those
  // launches are latency bound and independent, so they run concurrently on
  // side streams forked from and joined back to st.  Full phases run in
  // order on st (concurrent full launches compete for LDS and lose).
  const bool fan = phase == 1;
  // packed tables: this phase's list of sources whose sums do not fit starts empty
  if (TM == kTabPacked && E0.unfit_rec) LP_HIP(hipMemsetAsync(E0.unfit_count, 0, 4, st));
  if (fan) {
    if (!w.fork) {
      LP_HIP(hipEventCreateWithFlags(&w.fork, hipEventDisableTiming));
      for (int j = 0; j < Workspace::kSide; j++) {
        LP_HIP(hipStreamCreateWithFlags(&w.side[j], hipStreamNonBlocking));
        LP_HIP(hipEventCreateWithFlags(&w.join[j], hipEventDisableTiming));
      }
    }
    LP_HIP(hipEventRecord(w.fork, st));
    for (int j = 0; j < Workspace::kSide; j++) LP_HIP(hipStreamWaitEvent(w.side[j], w.fork, 0));
  }
  int turn = 0;
  // largest buckets first: their long-running workgroups start early
  for (int b = kBuckets - 1; b >= 0; b--) {
    WorkList wl{lists + (uint64_t)b * list_stride + (first ? first[b] : 0u), counts_host[b], stride, phase};
    const uint64_t items = items_of(b);
    if (items == 0) continue;
    Emit E = E0;
    E.work = work + (fan ? kSampledWork : 0) + b * 8;
    const int k = fan ? turn++ % (Workspace::kSide + 1) : 0;
    hipStream_t sb = k == 0 ? st : w.side[k - 1];
    const int slot = fan ? LaunchClock::kSlots + b : b;
    if (kept && b <= kBucketMid1) {
      // (not timed with the bucket: its clock covers the accumulation kernel)
      SrcRec* dst = kept + kept_off[b];
      hipLaunchKernelGGL(prune_weighted_kernel, dim3(grid_for(items, kPruneTile, (unsigned)num_cus() * 8)), dim3(256),
                         0, sb, gv, E, wl, dst, kept_count + b);
      LP_HIP(hipGetLastError());
      wl = WorkList{dst, 0, 1, 0, kept_count + b};
    }
    if (clk) LP_TRY(clk->start(slot, sb));
    if constexpr (!kQuery) {
      if (fan) {
        if (b == kBucketHuge)
          LP_TRY((launch_spa<kW, kQuery, true>(g, w, gv, E, wl, SpaItem{nullptr, nullptr, 0, 0}, items, sb)));
        else
          LP_TRY((launch_bucket<TM, kQuery, true>(g, b, gv, E, wl, items, sb)));
        if (clk) LP_TRY(clk->stop(slot, sb));
        continue;
      }
    }
    if (b == kBucketHuge) {
      LP_TRY((launch_spa<kW, kQuery, false>(g, w, gv, E, wl, SpaItem{nullptr, nullptr, 0, 0}, items, sb)));
    } else {
      LP_TRY((launch_bucket<TM, kQuery, false>(g, b, gv, E, wl, items, sb)));
    }
    if (clk) LP_TRY(clk->stop(slot, sb));
  }
  if (fan) {
    for (int j = 0; j < Workspace::kSide; j++) {
      LP_HIP(hipEventRecord(w.join[j], w.side[j]));
      LP_HIP(hipStreamWaitEvent(st, w.join[j], 0));
    }
  }
  if constexpr (TM == kTabPacked && !kQuery) {
    if (E0.unfit_rec) {
      // the sources handed over for sums too wide for a packed slot, with
      // 12-byte tables and the same fraction bits; the list's length is read
      // on the device, so no round trip precedes the launch
      Emit E = E0;
      E.unfit_rec = nullptr;
      E.work = work + (fan ? kSampledWork : 0) + (kStatRows - 1) * 8;
      WorkList wl{static_cast<const SrcRec*>(E0.unfit_rec), 0, 1, 0, E0.unfit_count};
      const int slot = (fan ? LaunchClock::kSlots : 0) + kBuckets + 1;
      if (clk) LP_TRY(clk->start(slot, st));
      if (fan)
        hipLaunchKernelGGL((acc_lds_kernel<1024, 1024, 7680, kTabSplit, false, 64, true>),
                           dim3((unsigned)num_cus() * 2), dim3(1024), 0, st, gv, E, wl);
      else
        hipLaunchKernelGGL((acc_lds_kernel<1024, 1024, 7680, kTabSplit, false, 64, false>),
                           dim3((unsigned)num_cus() * 2), dim3(1024), 0, st, gv, E, wl);
      LP_HIP(hipGetLastError());
      if (clk) LP_TRY(clk->stop(slot, st));
    }
  }
  // overflow records written by this phase's LDS kernels (and, in the same
  // round trip, the candidate count when the caller wants it)
  uint32_t ovf_total = 0;
  PinnedReads reads(w);
  LP_TRY(reads.add(&ovf_total, E0.ovf_count, 4, st));
  if (rb) LP_TRY(rb->issue(reads, st));
  LP_TRY(reads.finish(st));
  if (ovf_total > E0.ovf_cap) return set_error(LP_ERR_OUT_OF_MEMORY, "overflow list exhausted");
  if (ovf_total > *ovf_host_count) {
    WorkList none{nullptr, 0, 1, 0};
    SpaItem ov{E0.ovf, static_cast<const SrcRec*>(E0.ovf_rec), *ovf_host_count, ovf_total};
    Emit E = E0;
    E.work = work + kBucketHuge * 8;
    if (clk) LP_TRY(clk->start(kBuckets, st));
    LP_TRY((launch_spa<kW, kQuery, false>(g, w, gv, E, none, ov, ovf_total - *ovf_host_count, st)));
    if (clk) LP_TRY(clk->stop(kBuckets, st));
    *ovf_host_count = ovf_total;
    if (rb) LP_TRY(rb->issue(reads, st));
    LP_TRY(reads.finish(st));
  }
  if (clk) clk->collect();
  return LP_OK;
}

template <bool kQuery>
static lp_status run_phase_any(lp_graph* g, Workspace& w, const GView& gv, const Emit& E,
                               const SrcRec* lists, uint64_t list_stride,
                               const uint32_t* counts_host, uint32_t stride, int phase,
                               uint32_t* ovf_host_count, LaunchClock* clk, hipStream_t st,
                               const uint32_t* first = nullptr, const Readback* rb = nullptr,
                               bool prune = false) {
  // AA / RA: packed tables when the call set them up (pk_idbits > 0)
  if constexpr (!kQuery) {
    if ((E.measure == LP_AA || E.measure == LP_RA) && E.pk_idbits > 0)
      return run_phase<kTabPacked, kQuery>(g, w, gv, E, lists, list_stride, counts_host, stride, phase,
                                           ovf_host_count, clk, st, first, rb, prune);
  }
  if (E.measure == LP_AA || E.measure == LP_RA)
    return run_phase<kTabSplit, kQuery>(g, w, gv, E, lists, list_stride, counts_host, stride, phase,
                                        ovf_host_count, clk, st, first, rb, prune);
  return run_phase<kTabCount, kQuery>(g, w, gv, E, lists, list_stride, counts_host, stride, phase,
                                      ovf_host_count, clk, st, first, rb);
}

// Radix select of the k largest keys among entries [base, count) of the
// candidate buffer, into ws.tmp_*[1] ... the winners end in (os, oa, oc).
static lp_status run_select(lp_graph* g, const uint32_t* cs, const uint32_t* ca, const uint32_t* cc,
                            unsigned long long* count_dev, unsigned long long cap,
                            unsigned long long base, unsigned long long k, uint32_t* os,
                            uint32_t* oa, uint32_t* oc, uint32_t* tau_out, hipStream_t st,
                            bool full_key = false) {
  Workspace& w = g->ws;
  LP_TRY(w.sel_state.ensure(sizeof(SelState) + 64));
  LP_TRY(w.hist.ensure(2048 * 4));
  SelState* sst = w.sel_state.as<SelState>();
  uint32_t* hist = w.hist.as<uint32_t>();
  LP_HIP(hipMemsetAsync(hist, 0, 2048 * 4, st));
  hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(1), 0, st, sst, (const unsigned long long*)count_dev,
                     cap, base, k);
  LP_HIP(hipGetLastError());
  const unsigned cus = (unsigned)num_cus();
  const unsigned grid = cus * 4;
  const uint32_t* in_s = cs + base;
  const uint32_t* in_a = ca + base;
  const uint32_t* in_c = cc + base;
  hipLaunchKernelGGL(sel_copy_all_kernel, dim3(grid), dim3(256), 0, st, in_s, in_a, in_c, sst, os,
                     oa, oc);
  LP_HIP(hipGetLastError());
  int ping = 0;
  // a threshold estimate needs only the score digits: (score of the k-th key,
  // 0, 0) is a lower bound of the k-th key; full_key asks for the key itself
  const int nsteps = tau_out && !full_key ? 3 : 9;
  for (int step = 0; step < nsteps; step++) {
    uint32_t* nxt_s = w.tmp_s[ping].as<uint32_t>();
    uint32_t* nxt_a = w.tmp_a[ping].as<uint32_t>();
    uint32_t* nxt_c = w.tmp_c[ping].as<uint32_t>();
    hipLaunchKernelGGL(sel_hist_kernel, dim3(grid), dim3(256), 0, st, in_s, in_a, in_c, sst, step,
                       hist);
    hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(64), 0, st, sst, step, hist);
    hipLaunchKernelGGL(sel_partition_kernel, dim3(grid), dim3(256), 0, st, in_s, in_a, in_c, sst,
                       step, nxt_s, nxt_a, nxt_c, os, oa, oc);
    hipLaunchKernelGGL(sel_advance_kernel, dim3(1), dim3(1), 0, st, sst, step == nsteps - 1 ? 1 : 0);
    LP_HIP(hipGetLastError());
    in_s = nxt_s;
    in_a = nxt_a;
    in_c = nxt_c;
    ping ^= 1;
  }
  if (tau_out) {
    hipLaunchKernelGGL(sel_tau_kernel, dim3(1), dim3(1), 0, st, (const SelState*)sst, tau_out);
    LP_HIP(hipGetLastError());
  }
  return LP_OK;
}

static lp_status ensure_select_bufs(Workspace& w, uint64_t cap) {
  for (int i = 0; i < 2; i++) {
    LP_TRY(w.tmp_s[i].ensure(cap * 4));
    LP_TRY(w.tmp_a[i].ensure(cap * 4));
    LP_TRY(w.tmp_c[i].ensure(cap * 4));
  }
  return LP_OK;
}

// Sort (s desc, a asc, c asc) in place; id_bits bounds the a / c words.
static lp_status sort_keys(lp_graph* g, uint32_t* s, uint32_t* a, uint32_t* c, uint64_t k,
                           int a_bits, int c_bits, hipStream_t st) {
  Workspace& w = g->ws;
  SortSpec sp{};
  sp.w[0] = s;
  sp.w[1] = a;
  sp.w[2] = c;
  sp.nwords = 3;
  sp.nkeys = 3;
  sp.key_bits[0] = 32;
  sp.key_bits[1] = a_bits;
  sp.key_bits[2] = c_bits;
  sp.invert[0] = true;
  sp.invert[1] = false;
  sp.invert[2] = false;
  return radix_sort(sp, (int64_t)k, w.sort_tmp, w.sort_counts, w.scan_tmp, st);
}

static int id_bits(uint64_t n) {
  int b = 1;
  while (b < 32 && ((uint64_t)1 << b) < n) b++;
  return b;
}

struct PlanResult {
  PlanOut out;
  uint32_t hub;
};

static lp_status run_plan(lp_graph* g, int64_t L, PlanResult* pr, hipStream_t st) {
  Workspace& w = g->ws;
  const uint64_t n = (uint64_t)g->n;
  LP_TRY(w.lists.ensure(std::max<uint64_t>(n, 1) * sizeof(SrcRec) * kBuckets));
  LP_TRY(w.stats.ensure(sizeof(PlanOut) + 64));
  LP_TRY(w.host_stats.ensure(kHostStatsBytes));
  pr->hub = hub_start(g, L);
  const uint32_t hub_deg = L >= (int64_t)0xFFFFFFFE ? 0xFFFFFFFFu : (uint32_t)(L + 1);
  PlanOut* d_out = w.stats.as<PlanOut>();
  LP_HIP(hipMemsetAsync(d_out, 0, sizeof(PlanOut), st));
  const AccConfig cfg = acc_config(g);
  if (n > 0) {
    hipLaunchKernelGGL(plan_kernel, dim3(grid_for(n, 256 * kPlanItems, 0x7FFFFFFF)), dim3(256), 0, st,
                       view_of(g), hub_deg, cfg.cuts, w.lists.as<SrcRec>(), d_out);
    LP_HIP(hipGetLastError());
  }
  PlanOut* h = w.host_stats.as<PlanOut>();
  LP_HIP(hipMemcpyAsync(h, d_out, sizeof(PlanOut), hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  pr->out = *h;
  return LP_OK;
}

struct Timer {
  hipEvent_t* ev;
  explicit Timer(Workspace& w) : ev(workspace_events(w.timer_ev, 4)) {}
  float ms(int a, int b) {
    float t = 0;
    if (hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    return t;
  }
};

constexpr uint32_t kOvfCap = 1u << 16;  // overflow records of a call
constexpr size_t kCountersBytes = 4096 + (size_t)kOvfCap * (4 + sizeof(SrcRec));

// The counters block: call-wide counters in its first 4096 bytes (zeroed
// per call), then the overflow list.
static void ovf_layout(Workspace& w, uint32_t** ovf, void** ovf_rec, uint32_t** ovf_count, uint32_t* cap,
                       uint32_t** err, unsigned long long** count, unsigned long long** fp, uint32_t** tau) {
  const uint32_t ocap = kOvfCap;
  char* base = w.counters.as<char>();
  *count = reinterpret_cast<unsigned long long*>(base);   // [0]
  *fp = reinterpret_cast<unsigned long long*>(base + 64);  // [3]
  *ovf_count = reinterpret_cast<uint32_t*>(base + 128);
  *err = reinterpret_cast<uint32_t*>(base + 192);
  *tau = reinterpret_cast<uint32_t*>(base + 256);          // [3]
  *ovf = reinterpret_cast<uint32_t*>(base + 4096);
  *ovf_rec = base + 4096 + (size_t)ocap * 4;
  *cap = ocap;
}

static lp_status ensure_ovf(Workspace& w, uint32_t** ovf, void** ovf_rec, uint32_t** ovf_count,
                            uint32_t* cap, uint32_t** err, unsigned long long** count,
                            unsigned long long** fp, uint32_t** tau, hipStream_t st) {
  LP_TRY(w.counters.ensure(kCountersBytes));
  ovf_layout(w, ovf, ovf_rec, ovf_count, cap, err, count, fp, tau);
  LP_HIP(hipMemsetAsync(w.counters.p, 0, 4096, st));
  return LP_OK;
}

// Fraction bits of a call's AA / RA fixed-point sums: the most that keep every
// sum below 2^62 (a sum has at most max_deg terms, each at most 1/2 for RA
// and 1/ln 2 for AA), capped at 44.  A sum's relative rounding error is at most
// 2^-(F+1) / w_min, with w_min the weight of the largest explored degree; a
// call whose bound would exceed 2^-24 is refused rather than answered outside
// the 1e-6 tolerance.  That happens only for RA, when the largest explored
// degree times the maximum degree exceeds about 2^40.
static lp_status weighted_shift(const lp_graph* g, int m, int64_t L, int* shift) {
  *shift = g->fixed_shift;
  if (m != LP_AA && m != LP_RA) return LP_OK;
  const double wmax = m == LP_RA ? 0.5 : 1.0 / std::log(2.0);
  int F = 44;
  while (F > 0 && (double)(g->max_deg + 1) * wmax * std::ldexp(1.0, F) >= std::ldexp(1.0, 62)) F--;
  *shift = F;
  const uint32_t hs = hub_start(g, L);
  if (hs == 0) return LP_OK;
  const double dmax = (double)g->host_deg[hs - 1];
  if (dmax < 2.0) return LP_OK;
  const double inv_wmin = m == LP_RA ? dmax : std::log(dmax);
  if (std::ldexp(inv_wmin, -(F + 1)) > std::ldexp(1.0, -24))
    return set_error(LP_ERR_INVALID_ARGUMENT,
                     "%s sums in %d-bit fixed point cannot stay within 2^-24 of their value with "
                     "intermediates of degree %.0f (maximum degree %lld); use a lower hub limit",
                     m == LP_RA ? "RA" : "AA", F, dmax, (long long)g->max_deg);
  return LP_OK;
}

// Packed AA / RA tables for a prediction call (key and fixed-point sum in one
// 64-bit slot).  Every kernel and the global path of a call round the weights
// to the same F fraction bits, so results do not depend on which kernel a
// source lands in: F is what the tightest packed slot allows (48 sources of
// at most 32 arcs share a tiny batch: key bits id_bits(n + 1) + 6), at most
// the call's common shift.  Packing is used only when F keeps every sum within
// 2^-22 of its value: each term is rounded by at most 2^-(F+1) and no term is
// below the weight w_min of the largest explored degree, so F >= 21 +
// log2(1 / w_min) suffices.  Otherwise (or for other measures, or above
// 2^25 - 2 vertices) the call keeps 12-byte tables and its common shift.
static void packed_params(const lp_graph* g, int m, int64_t L, Emit* E) {
  E->pk_idbits = 0;
  if (m != LP_AA && m != LP_RA) return;
  const int ib = id_bits((uint64_t)g->n + 1);
  if (ib > 25) return;
  const uint32_t hs = hub_start(g, L);  // vertices of degree <= L form a prefix
  if (hs == 0) return;
  const double dmax = (double)g->host_deg[hs - 1];
  if (dmax < 2.0) return;
  const double inv_wmin = m == LP_RA ? dmax : std::log(dmax);
  const int fmin = 21 + std::max(0, (int)std::ceil(std::log2(inv_wmin)));
  const int e = m == LP_RA ? -1 : 1;
  const int ftiny = (63 - (ib + BatchKey<48>::kSrcBits)) - 1 - 5 - e;  // ceil(log2 32) = 5
  const int F = std::min(ftiny, E->shift);
  if (F < fmin) return;
  E->pk_idbits = ib;
  E->shift = F;
}

// The list of sources handed over by a packed call (SrcRec each, count
// first); empty for other calls.
static lp_status unfit_list(Workspace& w, Emit* E) {
  E->unfit_rec = nullptr;
  E->unfit_count = nullptr;
  E->unfit_cap = 0;
  if (E->pk_idbits == 0) return LP_OK;
  const uint32_t cap = 1u << 16;
  LP_TRY(w.unfit.ensure(256 + (size_t)cap * sizeof(SrcRec)));
  E->unfit_count = w.unfit.as<uint32_t>();
  E->unfit_rec = w.unfit.as<char>() + 256;
  E->unfit_cap = cap;
  return LP_OK;
}

// number of buffer entries whose key is >= tau
constexpr int kGeItems = 8;  // keys per thread per round of count_ge_kernel

// Number of keys >= tau.  Each round a block takes a contiguous tile of
// 256 * kGeItems keys with all of a thread's score loads in flight; the
// block's count reaches the global counter with one atomic (same-address
// atomics serialise, so their number is kept to the grid size).
__global__ __launch_bounds__(256) void count_ge_kernel(const uint32_t* __restrict__ ks,
                                                       const uint32_t* __restrict__ ka,
                                                       const uint32_t* __restrict__ kc,
                                                       unsigned long long n, const uint32_t* tau,
                                                       unsigned long long* out) {
  __shared__ unsigned long long part[4];
  const uint32_t t0 = tau[0], t1 = tau[1], t2 = tau[2];
  // a threshold (s, 0, 0) is met by every key of score >= s: the id words
  // are then never read
  const bool score_only = (t1 | t2) == 0;
  unsigned long long c = 0;
  for (unsigned long long base = (unsigned long long)blockIdx.x * (256 * kGeItems) + threadIdx.x;
       base < n; base += (unsigned long long)gridDim.x * (256 * kGeItems)) {
    uint32_t s[kGeItems];
#pragma unroll
    for (int j = 0; j < kGeItems; j++) {
      const unsigned long long i = base + (unsigned long long)j * 256;
      s[j] = i < n ? ks[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kGeItems; j++) {
      const unsigned long long i = base + (unsigned long long)j * 256;
      if (i >= n) continue;
      bool ge = s[j] > t0;
      if (s[j] == t0) {
        if (score_only) ge = true;
        else {
          const uint32_t a = ~ka[i], x = ~kc[i];
          ge = a > t1 || (a == t1 && x >= t2);
        }
      }
      c += ge ? 1ull : 0ull;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
  if (lane_id() == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = part[0] + part[1] + part[2] + part[3];
    if (t) atomicAdd(out, t);
  }
}

// Keys among the first n of the candidate buffer that are >= tau (read back).
static lp_status count_ge(Workspace& w, const Emit& E, unsigned long long n, const uint32_t* tau,
                          unsigned long long* out, hipStream_t st) {
  unsigned long long* ge = E.fp;  // scratch counter
  LP_HIP(hipMemsetAsync(ge, 0, 8, st));
  if (n > 0) {
    hipLaunchKernelGGL(count_ge_kernel, dim3(grid_for(n, 256 * kGeItems, num_cus() * 2)), dim3(256), 0, st,
                       E.out_s, E.out_a, E.out_c, n, tau, ge);
    LP_HIP(hipGetLastError());
  }
  PinnedReads reads(w);
  LP_TRY(reads.add(out, ge, 8, st));
  return reads.finish(st);
}

// A sampled threshold keeps only the score unless the keys tied with it
// would exceed this many times k.
constexpr unsigned long long kTieLimit = 3;
// The sample holds at least one in this many sources (of those with wedges).
constexpr uint64_t kMinSampleShare = 1024;

lp_status run_predict(lp_graph* g, int m, int64_t L, int64_t k, float s_th, int32_t* out_a,
                      int32_t* out_c, float* out_score, int64_t* out_count, hipStream_t st) {
  Workspace& w = g->ws;
  lp_stats& S = g->last;
  S = lp_stats{};
  *out_count = 0;
  Timer tm(w);
  LP_HIP(hipEventRecord(tm.ev[0], st));
  PlanResult pr;
  LP_TRY(run_plan(g, L, &pr, st));
  LP_HIP(hipEventRecord(tm.ev[1], st));
  S.wedges = pr.out.wedges;
  S.sources = pr.out.sources;
  for (int b = 0; b < kBuckets; b++) S.bucket_sources[b] = pr.out.count[b];
  const GView gv = view_of(g);
  uint32_t *ovf, *ovf_count, *err, *tau;
  void* ovf_rec;
  unsigned long long *count, *fp;
  uint32_t ovf_cap;
  LP_TRY(ensure_ovf(w, &ovf, &ovf_rec, &ovf_count, &ovf_cap, &err, &count, &fp, &tau, st));
  if (k == 0 || pr.out.wedges == 0 || g->n == 0) {
    LP_HIP(hipEventRecord(tm.ev[2], st));
    LP_HIP(hipEventRecord(tm.ev[3], st));
    LP_HIP(hipStreamSynchronize(st));
    S.ms_plan = tm.ms(0, 1);
    S.ms_total = tm.ms(0, 3);
    return LP_OK;
  }
  // the fixed-point precision bound of AA / RA is checked before any buffer
  // is sized from the wedge count
  int wshift = 0;
  LP_TRY(weighted_shift(g, m, L, &wshift));
  const uint64_t total_w = pr.out.wedges;
  const uint64_t budget = sample_budget(g, total_w);
  // Sampling pays off only when candidates far outnumber k: a sampled subset
  // of sources (every stride-th of each bucket) is scored first, without a
  // threshold; tau is then a lower bound of its r-th best key with
  // r = 1.5 k / stride, and the remaining sources only keep keys >= tau.
  const bool sample = budget > 0 && total_w > budget && total_w > 8ull * (uint64_t)k;
  // The stride also keeps at least one in kMinSampleShare sources in the
  // sample: with few hub intermediates cut (IBase, large L) the wedge budget
  // alone left a few dozen sampled sources, which miss the hubs that own the
  // best pairs, so the estimated threshold fell far too low and the main
  // pass overflowed its buffer.
  uint32_t stride = 1;
  if (sample) {
    const uint64_t s = (total_w + budget - 1) / budget;
    const uint64_t by_sources = std::max<uint64_t>(pr.out.sources / kMinSampleShare, 2);
    stride = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(std::max<uint64_t>(s, 2), by_sources), 1u << 20);
  }
  uint64_t cap = sample ? 2 * (total_w / stride) + 4 * (uint64_t)k + (1u << 20) : total_w;
  cap = std::min<uint64_t>(cap, total_w);
  cap = std::min<uint64_t>(cap, (1ull << 32) - 1);
  const uint64_t kcap = std::min<uint64_t>((uint64_t)k, cap);
  LP_TRY(w.cand_s.ensure(cap * 4));
  LP_TRY(w.cand_a.ensure(cap * 4));
  LP_TRY(w.cand_c.ensure(cap * 4));
  LP_TRY(ensure_select_bufs(w, cap));
  LP_TRY(w.q_out.ensure(kcap * 12 + 64));
  LP_TRY(w.q_cnt.ensure(cap * 12 + 64));  // outputs of the threshold selections
  uint32_t* os = w.q_out.as<uint32_t>();
  uint32_t* oa = os + kcap;
  uint32_t* oc = oa + kcap;
  uint32_t* ts = w.q_cnt.as<uint32_t>();
  uint32_t* ta = ts + cap;
  uint32_t* tc = ta + cap;
  Emit E{};
  E.measure = m;
  E.shift = wshift;
  E.s_th = s_th;
  E.tau = tau;
  packed_params(g, m, L, &E);
  LP_TRY(unfit_list(w, &E));
  E.out_s = w.cand_s.as<uint32_t>();
  E.out_a = w.cand_a.as<uint32_t>();
  E.out_c = w.cand_c.as<uint32_t>();
  E.out_count = count;
  E.cap = cap;
  E.fp = fp;
  E.ovf = ovf;
  E.ovf_rec = ovf_rec;
  E.ovf_count = ovf_count;
  E.ovf_cap = ovf_cap;
  E.err = err;
  const SrcRec* lists = w.lists.as<SrcRec>();
  uint32_t ovf_host = 0;
  unsigned long long n_sample = 0;
  LaunchClock clk(&S, w);
  if (sample) {
    Readback rb;
    rb.dst[0] = &n_sample;
    rb.src[0] = count;
    rb.bytes[0] = 8;
    LP_TRY(run_phase_any<false>(g, w, gv, E, lists, (uint64_t)g->n, pr.out.count,
                                stride, 1, &ovf_host, &clk, st, nullptr, &rb));
    if (n_sample > cap) return set_error(LP_ERR_OUT_OF_MEMORY, "sample exceeded its buffer");
  }
  unsigned long long r_target =
      (unsigned long long)std::ceil(1.5 * (double)k / (double)stride) + 64;
  bool need_tau = sample;
  for (uint64_t retries = 0;; retries++) {
    if (retries > 40) return set_error(LP_ERR_DEVICE, "top-k threshold did not converge");
    if (sample) {
      // drop the previous pass's appends (the count is n_sample already on
      // the first pass: it was read back from there)
      if (retries > 0) LP_HIP(hipMemcpyAsync(count, &n_sample, 8, hipMemcpyHostToDevice, st));
      if (need_tau) {
        if (r_target >= n_sample) LP_HIP(hipMemsetAsync(tau, 0, 12, st));
        else {
          LP_TRY(run_select(g, E.out_s, E.out_a, E.out_c, count, cap, 0, r_target, ts, ta, tc, tau, st));
          // The score alone admits every key tied with the r-th one.  With
          // integer-like scores (CN at small hub limits) that run can hold
          // many times k keys, overflow the buffer and force a second pass;
          // then a key of the sample itself (score and ids) is the bound,
          // taken twice as deep (about 3 k keys): which sources the sample
          // holds varies with the order of the bucket lists, and a tied run
          // that a few sources dominate makes the ids' estimate noisy.
          unsigned long long nge = 0;
          LP_TRY(count_ge(w, E, n_sample, tau, &nge, st));
          const unsigned long long r_full = 2 * r_target;
          if (nge * (unsigned long long)stride > kTieLimit * (unsigned long long)k && r_full < n_sample)
            LP_TRY(run_select(g, E.out_s, E.out_a, E.out_c, count, cap, 0, r_full, ts, ta, tc, tau, st,
                              true));
        }
      }
    }
    unsigned long long n_total = 0;
    uint32_t tau_h[3] = {0, 0, 0};
    Readback rb;
    rb.dst[0] = &n_total;
    rb.src[0] = count;
    rb.bytes[0] = 8;
    rb.dst[1] = tau_h;
    rb.src[1] = tau;
    rb.bytes[1] = 12;
    if (sample)
      LP_TRY(run_phase_any<false>(g, w, gv, E, lists, (uint64_t)g->n, pr.out.count,
                                  stride, 2, &ovf_host, &clk, st, nullptr, &rb, true));
    else
      LP_TRY(run_phase_any<false>(g, w, gv, E, lists, (uint64_t)g->n, pr.out.count,
                                  1, 0, &ovf_host, &clk, st, nullptr, &rb));
    if (retries == 0) LP_HIP(hipEventRecord(tm.ev[2], st));
    if (n_total > cap) {
      if (!sample)
        return set_error(LP_ERR_OUT_OF_MEMORY, "candidate buffer overflow (%llu > %llu)",
                         (unsigned long long)n_total, (unsigned long long)cap);
      // the buffer holds >= k real candidates: its k-th best key (in full,
      // since the score alone does not separate ties) is a safe tau
      LP_TRY(run_select(g, E.out_s, E.out_a, E.out_c, count, cap, 0, (unsigned long long)k, ts, ta,
                        tc, tau, st, true));
      need_tau = false;
      continue;
    }
    const bool tau_zero = (tau_h[0] | tau_h[1] | tau_h[2]) == 0;
    if (!tau_zero) {
      // every candidate >= tau is in the buffer; the answer is there iff
      // at least k of them are
      unsigned long long nge = 0;
      LP_TRY(count_ge(w, E, n_total, tau, &nge, st));
      if (nge < (unsigned long long)k) {
        r_target = r_target >= n_sample / 4 ? n_sample : r_target * 4;
        need_tau = true;
        continue;
      }
    }
    S.appended = n_total;
    S.retries = retries;
    LP_TRY(run_select(g, E.out_s, E.out_a, E.out_c, count, cap, 0, (unsigned long long)k, os, oa, oc,
                      nullptr, st));
    // the select emits min(k, n_total) keys; its own count is checked in the
    // call's last round trip
    const uint64_t kout = std::min<uint64_t>((uint64_t)k, n_total);
    LP_TRY(sort_keys(g, os, oa, oc, kout, id_bits((uint64_t)g->n), id_bits((uint64_t)g->n), st));
    LP_HIP(hipEventRecord(tm.ev[3], st));
    hipPointerAttribute_t at;
    const bool dev_out =
        hipPointerGetAttributes(&at, out_a) == hipSuccess && at.type == hipMemoryTypeDevice &&
        hipPointerGetAttributes(&at, out_c) == hipSuccess && at.type == hipMemoryTypeDevice &&
        hipPointerGetAttributes(&at, out_score) == hipSuccess && at.type == hipMemoryTypeDevice;
    (void)hipGetLastError();
    if (kout > 0) {
      if (dev_out) {
        hipLaunchKernelGGL(write_out_kernel, dim3(grid_for(kout, 256, 65536)), dim3(256), 0, st, os,
                           oa, oc, (unsigned long long)kout, out_a, out_c, out_score);
        LP_HIP(hipGetLastError());
      } else {
        int32_t* xa = reinterpret_cast<int32_t*>(ts);
        int32_t* xc = xa + kout;
        float* xs = reinterpret_cast<float*>(xc + kout);
        hipLaunchKernelGGL(write_out_kernel, dim3(grid_for(kout, 256, 65536)), dim3(256), 0, st, os,
                           oa, oc, (unsigned long long)kout, xa, xc, xs);
        LP_HIP(hipGetLastError());
        LP_HIP(hipMemcpyAsync(out_a, xa, kout * 4, hipMemcpyDefault, st));
        LP_HIP(hipMemcpyAsync(out_c, xc, kout * 4, hipMemcpyDefault, st));
        LP_HIP(hipMemcpyAsync(out_score, xs, kout * 4, hipMemcpyDefault, st));
      }
    }
    SelState hs;
    uint32_t herr = 0;
    unsigned long long wk[2 * kSampledWork];
    PinnedReads reads(w);
    LP_TRY(reads.add(&hs, w.sel_state.p, sizeof(SelState), st));
    LP_TRY(reads.add(&herr, err, 4, st));
    LP_TRY(reads.add(wk, work_counters(w), sizeof(wk), st));
    LP_TRY(reads.finish(st));
    if (hs.n_out != kout)
      return set_error(LP_ERR_DEVICE, "selection returned %llu of %llu keys", hs.n_out,
                       (unsigned long long)kout);
    if (herr) return set_error(LP_ERR_DEVICE, "device error flags 0x%x", herr);
    *out_count = (int64_t)kout;
    fill_work(wk, &S);
    S.ms_plan = tm.ms(0, 1);
    S.ms_accumulate = tm.ms(1, 2);
    S.ms_select = tm.ms(2, 3);
    S.ms_total = tm.ms(0, 3);
    return LP_OK;
  }
}

// ---------------------------------------------------------------------------
// Several graphs in one call.  The resident graph is the disjoint union of
// ngraphs graphs, graph i owning original ids [gstart[i], gstart[i+1]).  Every
// accumulation launch covers all graphs (no two-hop path leaves a graph, so
// candidates never mix); thresholds and the final top-k are per graph.
// ---------------------------------------------------------------------------

__device__ inline uint32_t graph_of_id(const uint32_t* gstart, uint32_t ng, uint32_t key) {
  uint32_t lo = 0, hi = ng;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (gstart[mid] <= key) lo = mid;
    else hi = mid;
  }
  return lo;
}

// err |= 1 if an edge joins two graphs
__global__ void cross_check_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                                   const uint32_t* __restrict__ rank, const uint32_t* __restrict__ perm,
                                   const uint32_t* __restrict__ gstart, uint32_t ng, int64_t n,
                                   uint32_t* err) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const uint32_t gi = graph_of_id(gstart, ng, (uint32_t)o);
  const uint32_t lo = gstart[gi], hi = gstart[gi + 1];
  const uint32_t v = rank[o];
  bool bad = false;
  for (uint32_t e = off[v]; e < off[v + 1]; e++) {
    const uint32_t b = perm[adj[e]];
    bad = bad || b < lo || b >= hi;
  }
  if (bad) atomicOr(err, 1u);
}

// Per-graph histograms of the kernels below: in LDS while the graphs fit
// (flushed once per workgroup), else straight to global memory.  The graph
// boundaries are staged in LDS alongside.
constexpr uint32_t kGraphLds = 2048;

struct GraphLds {
  uint32_t start[kGraphLds + 1];
  uint32_t hist[kGraphLds];
};

__device__ inline const uint32_t* graph_lds_init(GraphLds& L, const uint32_t* gstart, uint32_t ng) {
  const bool lds = ng <= kGraphLds;
  if (lds)
    for (uint32_t t = threadIdx.x; t <= ng; t += blockDim.x) {
      L.start[t] = gstart[t];
      if (t < ng) L.hist[t] = 0;
    }
  __syncthreads();
  return lds ? L.start : gstart;
}

// graph id of each candidate (by its smaller original id) and per-graph counts
__global__ __launch_bounds__(256) void graph_id_kernel(const uint32_t* __restrict__ a, unsigned long long n,
                                                       const uint32_t* __restrict__ gstart, uint32_t ng,
                                                       uint32_t* __restrict__ gid, uint32_t* __restrict__ gcount) {
  __shared__ GraphLds L;
  const bool lds = ng <= kGraphLds;
  const uint32_t* gs = graph_lds_init(L, gstart, ng);
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t gi = graph_of_id(gs, ng, a[i]);
    gid[i] = gi;
    atomicAdd(lds ? &L.hist[gi] : &gcount[gi], 1u);
  }
  __syncthreads();
  if (lds)
    for (uint32_t t = threadIdx.x; t < ng; t += blockDim.x)
      if (L.hist[t]) atomicAdd(&gcount[t], L.hist[t]);
}

// murmur3's 32-bit finaliser: spreads the original ids for the sample draw
__device__ inline uint32_t sample_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  x *= 0xC2B2AE35u;
  x ^= x >> 16;
  return x;
}

// Split one bucket list by each source's graph sampling stride: a source is
// in the sample when the hash of its original id is a multiple of the stride.
// The rest fill out[0, rest) and the sample fills out[count - sampled, count)
// (from the top down); ctr[0] / ctr[1] count them.  One pair of atomics per
// tile of 1024 records.
constexpr int kSplitRounds = 4;

__global__ __launch_bounds__(256) void graph_split_kernel(const SrcRec* __restrict__ in, uint32_t count,
                                                          const uint32_t* __restrict__ gstart, uint32_t ng,
                                                          const uint32_t* __restrict__ gstride,
                                                          SrcRec* __restrict__ out, uint32_t* __restrict__ ctr,
                                                          unsigned long long* __restrict__ sampled_wedges) {
  __shared__ uint32_t cnt[kSplitRounds][4][2];
  __shared__ uint32_t base[2];
  __shared__ unsigned long long wsum[4];
  unsigned long long my_w = 0;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  constexpr uint64_t kTile = 256ull * kSplitRounds;
  for (uint64_t t0 = (uint64_t)blockIdx.x * kTile; t0 < count; t0 += (uint64_t)gridDim.x * kTile) {
    SrcRec r[kSplitRounds];
    bool valid[kSplitRounds], samp[kSplitRounds];
    uint64_t bs[kSplitRounds], br[kSplitRounds];
#pragma unroll
    for (int j = 0; j < kSplitRounds; j++) {
      const uint64_t i = t0 + (uint64_t)j * 256 + threadIdx.x;
      valid[j] = i < count;
      samp[j] = false;
      if (valid[j]) {
        r[j] = in[i];
        const uint32_t sd = gstride[graph_of_id(gstart, ng, r[j].key)];
        samp[j] = sd <= 1 || sample_hash(r[j].key) % sd == 0;
        if (samp[j]) my_w += r[j].U;
      }
      bs[j] = __ballot(valid[j] && samp[j]);
      br[j] = __ballot(valid[j] && !samp[j]);
      if (lane == 0) {
        cnt[j][wid][0] = (uint32_t)__popcll(br[j]);
        cnt[j][wid][1] = (uint32_t)__popcll(bs[j]);
      }
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      uint32_t tot = 0;
      for (int j = 0; j < kSplitRounds; j++)
        for (int w = 0; w < 4; w++) tot += cnt[j][w][threadIdx.x];
      base[threadIdx.x] = tot ? atomicAdd(&ctr[threadIdx.x], tot) : 0u;
    }
    __syncthreads();
    uint32_t pr = base[0], ps = base[1];
#pragma unroll
    for (int j = 0; j < kSplitRounds; j++) {
      uint32_t wr = 0, ws = 0;
      for (int w = 0; w < 4; w++) {
        if (w < wid) {
          wr += cnt[j][w][0];
          ws += cnt[j][w][1];
        }
      }
      if (valid[j]) {
        if (samp[j]) out[count - 1 - (ps + ws + (uint32_t)__popcll(bs[j] & lt))] = r[j];
        else out[pr + wr + (uint32_t)__popcll(br[j] & lt)] = r[j];
      }
      for (int w = 0; w < 4; w++) {
        pr += cnt[j][w][0];
        ps += cnt[j][w][1];
      }
    }
    __syncthreads();
  }
  for (int o = 32; o >= 1; o >>= 1) my_w += __shfl_xor(my_w, o);
  if (lane == 0) wsum[wid] = my_w;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (t) atomicAdd(sampled_wedges, t);
  }
}

// Per-graph threshold from the sample sorted by (graph, score desc): the
// score of the graph's r-th best sampled candidate with ids 0 (a lower bound
// of that key), r = 1.5 k / stride + 64 with the graph's sampling stride; no
// threshold when the graph sampled fewer; k = 0 keeps nothing.
__global__ void graph_tau_kernel(uint32_t ng, const uint32_t* __restrict__ gcount,
                                 const uint32_t* __restrict__ gseg, const uint32_t* __restrict__ s_sorted,
                                 const unsigned long long* __restrict__ gk,
                                 const uint32_t* __restrict__ gstride, uint32_t* __restrict__ gtau) {
  const uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= ng) return;
  const unsigned long long k = gk[gi];
  const unsigned long long stride = gstride[gi] > 0 ? gstride[gi] : 1;
  uint32_t t = 0;
  const bool none = k == 0;
  if (none) {
    t = 0x7F800000u;  // +inf: no finite score reaches it
  } else {
    const unsigned long long r = (3 * k + 2 * stride - 1) / (2 * stride) + 64;
    if (gcount[gi] >= r) t = s_sorted[gseg[gi] + r - 1];
  }
  gtau[3 * gi] = t;
  gtau[3 * gi + 1] = none ? 0xFFFFFFFFu : 0u;
  gtau[3 * gi + 2] = none ? 0xFFFFFFFFu : 0u;
}

// per-graph number of buffer entries whose key is >= the graph's threshold
__global__ __launch_bounds__(256) void graph_count_ge_kernel(
    const uint32_t* __restrict__ ks, const uint32_t* __restrict__ ka, const uint32_t* __restrict__ kc,
    unsigned long long n, const uint32_t* __restrict__ gstart, uint32_t ng,
    const uint32_t* __restrict__ gtau, unsigned long long* out) {
  __shared__ GraphLds L;
  const bool lds = ng <= kGraphLds;
  const uint32_t* gs = graph_lds_init(L, gstart, ng);
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t gi = graph_of_id(gs, ng, ka[i]);
    const uint32_t t0 = gtau[3 * gi], t1 = gtau[3 * gi + 1], t2 = gtau[3 * gi + 2];
    const uint32_t s = ks[i], a = ~ka[i], x = ~kc[i];
    if (s > t0 || (s == t0 && (a > t1 || (a == t1 && x >= t2)))) {
      if (lds) atomicAdd(&L.hist[gi], 1u);
      else atomicAdd(&out[gi], 1ull);
    }
  }
  __syncthreads();
  if (lds)
    for (uint32_t t = threadIdx.x; t < ng; t += blockDim.x)
      if (L.hist[t]) atomicAdd(&out[t], (unsigned long long)L.hist[t]);
}

// the first k_g entries of each graph's segment of the sorted buffer
__global__ void graph_take_kernel(const uint32_t* __restrict__ gid, const uint32_t* __restrict__ s,
                                  const uint32_t* __restrict__ a, const uint32_t* __restrict__ c,
                                  unsigned long long n, const uint32_t* __restrict__ gseg,
                                  const unsigned long long* __restrict__ gk,
                                  const unsigned long long* __restrict__ goff, int32_t* __restrict__ oa,
                                  int32_t* __restrict__ oc, float* __restrict__ os) {
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t gi = gid[i];
    const unsigned long long r = i - gseg[gi];
    if (r < gk[gi]) {
      const unsigned long long pos = goff[gi] + r;
      oa[pos] = (int32_t)a[i];
      oc[pos] = (int32_t)c[i];
      os[pos] = __uint_as_float(s[i]);
    }
  }
}

lp_status run_predict_multi(lp_graph* g, int64_t ng, const int64_t* vstart, const int64_t* kk, int m,
                            int64_t L, float s_th, int32_t* out_a, int32_t* out_c, float* out_score,
                            int64_t* out_count, hipStream_t st) {
  Workspace& w = g->ws;
  lp_stats& S = g->last;
  S = lp_stats{};
  for (int64_t i = 0; i < ng; i++) out_count[i] = 0;
  const uint32_t NG = (uint32_t)ng;
  // per-graph tables: gstart[ng+1] u32, gtau[3ng] u32, gcount[ng] u32, gseg[ng] u32,
  // gstride[ng] u32, split counters [2 kBuckets] u32, then gk[ng] u64,
  // goff[ng] u64, gge[ng] u64, sampled wedges u64
  uint64_t ktot = 0;
  std::vector<uint32_t> hstart(NG + 1);
  std::vector<unsigned long long> hk(NG), hoff(NG);
  for (uint32_t i = 0; i <= NG; i++) hstart[i] = (uint32_t)vstart[i];
  for (uint32_t i = 0; i < NG; i++) {
    hk[i] = (unsigned long long)kk[i];
    hoff[i] = ktot;
    ktot += hk[i];
  }
  const size_t u32n = ((size_t)NG + 1 + 3 * (size_t)NG + 3 * (size_t)NG + 2 * kBuckets + 63) & ~(size_t)63;
  LP_TRY(w.m_graph.ensure(u32n * 4 + (size_t)NG * 8 * 3 + 256));
  uint32_t* gstart = w.m_graph.as<uint32_t>();
  uint32_t* gtau = gstart + NG + 1;
  uint32_t* gcount = gtau + 3 * (size_t)NG;
  uint32_t* gseg = gcount + NG;
  uint32_t* gstride = gseg + NG;
  uint32_t* split_ctr = gstride + NG;
  unsigned long long* gk = reinterpret_cast<unsigned long long*>(w.m_graph.as<char>() + u32n * 4);
  unsigned long long* goff = gk + NG;
  unsigned long long* gge = goff + NG;
  unsigned long long* samp_w = gge + NG;
  LP_HIP(hipMemcpyAsync(gstart, hstart.data(), (NG + 1) * 4, hipMemcpyHostToDevice, st));
  LP_HIP(hipMemcpyAsync(gk, hk.data(), NG * 8, hipMemcpyHostToDevice, st));
  LP_HIP(hipMemcpyAsync(goff, hoff.data(), NG * 8, hipMemcpyHostToDevice, st));
  LP_HIP(hipMemsetAsync(gtau, 0, (size_t)NG * 12, st));
  uint32_t *ovf, *ovf_count, *err, *tau;
  void* ovf_rec;
  unsigned long long *count, *fp;
  uint32_t ovf_cap;
  LP_TRY(ensure_ovf(w, &ovf, &ovf_rec, &ovf_count, &ovf_cap, &err, &count, &fp, &tau, st));
  // the graph never changes: a layout checked once stays valid
  if (g->n > 0 && w.m_checked != hstart) {
    hipLaunchKernelGGL(cross_check_kernel, dim3(grid_for((uint64_t)g->n, 256, 0x7FFFFFFF)), dim3(256), 0,
                       st, g->off, g->adj, g->rank, g->perm, gstart, NG, g->n, err);
    LP_HIP(hipGetLastError());
    uint32_t herr = 0;
    LP_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    if (herr) return set_error(LP_ERR_INVALID_GRAPH, "an edge joins two of the graphs");
    w.m_checked = hstart;
  }
  Timer tm(w);
  LP_HIP(hipEventRecord(tm.ev[0], st));
  PlanResult pr;
  LP_TRY(run_plan(g, L, &pr, st));
  LP_HIP(hipEventRecord(tm.ev[1], st));
  S.wedges = pr.out.wedges;
  S.sources = pr.out.sources;
  for (int b = 0; b < kBuckets; b++) S.bucket_sources[b] = pr.out.count[b];
  if (ktot == 0 || pr.out.wedges == 0) {
    LP_HIP(hipStreamSynchronize(st));
    return LP_OK;
  }
  const GView gv = view_of(g);
  // the fixed-point precision bound of AA / RA is checked before any buffer
  // is sized from the wedge count
  int wshift = 0;
  LP_TRY(weighted_shift(g, m, L, &wshift));
  const uint64_t total_w = pr.out.wedges;
  const uint64_t budget = sample_budget(g, total_w);
  const bool sample = budget > 0 && total_w > budget && total_w > 8ull * ktot;
  uint32_t stride = 1;
  const unsigned cus = (unsigned)num_cus();
  const SrcRec* lists = w.lists.as<SrcRec>();
  const uint64_t nl = (uint64_t)g->n;  // list stride of the bucket lists
  // With sampling, every graph draws its own sample: the global stride
  // W / budget, but at least one source in n_i / kMinSampled for a graph of
  // n_i vertices (every source of a small one), so that each threshold rests
  // on many sources.  The bucket lists are split into the sample and the
  // rest (w.m_lists).
  constexpr uint64_t kMinSampled = 256;
  uint32_t first[kBuckets] = {}, n_samp[kBuckets] = {}, n_rest[kBuckets] = {};
  unsigned long long samp_wedges = 0;
  const SrcRec* split_lists = nullptr;
  if (sample) {
    const uint64_t sd = (total_w + budget - 1) / budget;
    stride = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(sd, 2), 1u << 20);
    std::vector<uint32_t> hsd(NG);
    for (uint32_t i = 0; i < NG; i++)
      hsd[i] = (uint32_t)std::max<uint64_t>(
          1, std::min<uint64_t>(stride, (uint64_t)(hstart[i + 1] - hstart[i]) / kMinSampled));
    LP_HIP(hipMemcpyAsync(gstride, hsd.data(), (size_t)NG * 4, hipMemcpyHostToDevice, st));
    LP_TRY(w.m_lists.ensure(std::max<uint64_t>(nl, 1) * sizeof(SrcRec) * kBuckets));
    LP_HIP(hipMemsetAsync(split_ctr, 0, 2 * kBuckets * 4, st));
    LP_HIP(hipMemsetAsync(samp_w, 0, 8, st));
    for (int b = 0; b < kBuckets; b++) {
      if (pr.out.count[b] == 0) continue;
      hipLaunchKernelGGL(graph_split_kernel,
                         dim3(grid_for(pr.out.count[b], 256 * kSplitRounds, cus * 4)), dim3(256), 0, st,
                         lists + (uint64_t)b * nl, pr.out.count[b], gstart, NG, gstride,
                         w.m_lists.as<SrcRec>() + (uint64_t)b * nl, split_ctr + 2 * b, samp_w);
      LP_HIP(hipGetLastError());
    }
    uint32_t hc[2 * kBuckets];
    LP_HIP(hipMemcpyAsync(hc, split_ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
    LP_HIP(hipMemcpyAsync(&samp_wedges, samp_w, 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < kBuckets; b++) {
      n_rest[b] = hc[2 * b];
      n_samp[b] = hc[2 * b + 1];
      if (n_rest[b] + n_samp[b] != pr.out.count[b]) return set_error(LP_ERR_DEVICE, "list split lost records");
      first[b] = pr.out.count[b] - n_samp[b];
    }
    split_lists = w.m_lists.as<SrcRec>();
  }
  // the sample keeps every candidate of its sources (at most its wedges)
  uint64_t cap = sample ? samp_wedges + 4 * ktot + (1u << 20) : total_w;
  cap = std::min<uint64_t>(cap, total_w);
  cap = std::min<uint64_t>(cap, (1ull << 32) - 1);
  LP_TRY(w.cand_s.ensure(cap * 4));
  LP_TRY(w.cand_a.ensure(cap * 4));
  LP_TRY(w.cand_c.ensure(cap * 4));
  LP_TRY(w.m_gid.ensure(cap * 4));
  LP_TRY(ensure_select_bufs(w, cap));
  Emit E{};
  E.measure = m;
  E.shift = wshift;
  E.s_th = s_th;
  E.tau = tau;
  packed_params(g, m, L, &E);
  LP_TRY(unfit_list(w, &E));
  E.out_s = w.cand_s.as<uint32_t>();
  E.out_a = w.cand_a.as<uint32_t>();
  E.out_c = w.cand_c.as<uint32_t>();
  E.out_count = count;
  E.cap = cap;
  E.fp = fp;
  E.ovf = ovf;
  E.ovf_rec = ovf_rec;
  E.ovf_count = ovf_count;
  E.ovf_cap = ovf_cap;
  E.err = err;
  E.gtau = gtau;
  E.gstart = gstart;
  E.ngraphs = NG;
  uint32_t ovf_host = 0;
  unsigned long long n_sample = 0;
  LaunchClock clk(&S, w);
  uint32_t* gid = w.m_gid.as<uint32_t>();
  if (sample) {
    // sampled sources without thresholds, then each graph's threshold
    Readback rb;
    rb.dst[0] = &n_sample;
    rb.src[0] = count;
    rb.bytes[0] = 8;
    LP_TRY(run_phase_any<false>(g, w, gv, E, split_lists, nl, n_samp, 1, 1, &ovf_host, &clk, st, first, &rb));
    if (n_sample > cap) return set_error(LP_ERR_OUT_OF_MEMORY, "sample exceeded its buffer");
    LP_HIP(hipMemsetAsync(gcount, 0, (size_t)NG * 4, st));
    uint32_t* ts = w.tmp_s[0].as<uint32_t>();
    uint32_t* tg = w.tmp_a[0].as<uint32_t>();
    if (n_sample > 0) {
      hipLaunchKernelGGL(graph_id_kernel, dim3(grid_for(n_sample, 256, cus * 8)), dim3(256), 0, st,
                         E.out_a, n_sample, gstart, NG, tg, gcount);
      LP_HIP(hipGetLastError());
      LP_HIP(hipMemcpyAsync(ts, E.out_s, n_sample * 4, hipMemcpyDeviceToDevice, st));
      SortSpec sp{};
      sp.w[0] = tg;
      sp.w[1] = ts;
      sp.nwords = 2;
      sp.nkeys = 2;
      sp.key_bits[0] = id_bits(NG);
      sp.key_bits[1] = 32;
      sp.invert[1] = true;
      LP_TRY(radix_sort(sp, (int64_t)n_sample, w.sort_tmp, w.sort_counts, w.scan_tmp, st));
    }
    LP_TRY(scan_exclusive_u32(gcount, gseg, (int64_t)NG, w.scan_tmp, st));
    hipLaunchKernelGGL(graph_tau_kernel, dim3((NG + 255) / 256), dim3(256), 0, st, NG, gcount, gseg, ts,
                       gk, gstride, gtau);
    LP_HIP(hipGetLastError());
  }
  unsigned long long n_total = 0;
  for (int attempt = 0;; attempt++) {
    if (attempt > 4) return set_error(LP_ERR_DEVICE, "per-graph thresholds did not converge");
    Readback rb;
    rb.dst[0] = &n_total;
    rb.src[0] = count;
    rb.bytes[0] = 8;
    if (sample) {
      LP_HIP(hipMemcpyAsync(count, &n_sample, 8, hipMemcpyHostToDevice, st));
      LP_TRY(run_phase_any<false>(g, w, gv, E, split_lists, nl, n_rest, 1, 0, &ovf_host, &clk, st, nullptr,
                                  &rb, true));
    } else {
      LP_TRY(run_phase_any<false>(g, w, gv, E, lists, (uint64_t)g->n, pr.out.count, 1, 0, &ovf_host,
                                  &clk, st, nullptr, &rb));
    }
    if (n_total > cap) {
      // graphs without a threshold kept more than the buffer holds: the pass
      // counted every entry, so grow to that and run it again
      if (n_total >= (1ull << 32) - 1)
        return set_error(LP_ERR_OUT_OF_MEMORY, "candidate buffer overflow (%llu)",
                         (unsigned long long)n_total);
      const uint64_t ncap = n_total;
      const unsigned long long keep = sample ? n_sample : 0;
      if (keep > 0) {  // the sampled entries move with the buffers
        LP_TRY(w.tmp_s[1].ensure(keep * 4));
        LP_TRY(w.tmp_a[1].ensure(keep * 4));
        LP_TRY(w.tmp_c[1].ensure(keep * 4));
        LP_HIP(hipMemcpyAsync(w.tmp_s[1].p, E.out_s, keep * 4, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipMemcpyAsync(w.tmp_a[1].p, E.out_a, keep * 4, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipMemcpyAsync(w.tmp_c[1].p, E.out_c, keep * 4, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipStreamSynchronize(st));
      }
      w.cand_s.release();
      w.cand_a.release();
      w.cand_c.release();
      LP_TRY(w.cand_s.ensure(ncap * 4));
      LP_TRY(w.cand_a.ensure(ncap * 4));
      LP_TRY(w.cand_c.ensure(ncap * 4));
      LP_TRY(w.m_gid.ensure(ncap * 4));
      if (keep > 0) {
        LP_HIP(hipMemcpyAsync(w.cand_s.p, w.tmp_s[1].p, keep * 4, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipMemcpyAsync(w.cand_a.p, w.tmp_a[1].p, keep * 4, hipMemcpyDeviceToDevice, st));
        LP_HIP(hipMemcpyAsync(w.cand_c.p, w.tmp_c[1].p, keep * 4, hipMemcpyDeviceToDevice, st));
      }
      cap = ncap;
      E.cap = cap;
      E.out_s = w.cand_s.as<uint32_t>();
      E.out_a = w.cand_a.as<uint32_t>();
      E.out_c = w.cand_c.as<uint32_t>();
      gid = w.m_gid.as<uint32_t>();
      if (!sample) LP_HIP(hipMemsetAsync(count, 0, 8, st));
      S.retries++;
      continue;
    }
    if (!sample) break;
    // a graph's answer is in the buffer iff at least k of its keys are >= its threshold
    LP_HIP(hipMemsetAsync(gge, 0, (size_t)NG * 8, st));
    hipLaunchKernelGGL(graph_count_ge_kernel, dim3(grid_for(n_total, 256, cus * 8)), dim3(256), 0, st,
                       E.out_s, E.out_a, E.out_c, n_total, gstart, NG, gtau, gge);
    LP_HIP(hipGetLastError());
    std::vector<unsigned long long> hge(NG);
    std::vector<uint32_t> htau(3 * (size_t)NG);
    LP_HIP(hipMemcpyAsync(hge.data(), gge, NG * 8, hipMemcpyDeviceToHost, st));
    LP_HIP(hipMemcpyAsync(htau.data(), gtau, NG * 12, hipMemcpyDeviceToHost, st));
    LP_HIP(hipStreamSynchronize(st));
    bool redo = false;
    for (uint32_t i = 0; i < NG; i++) {
      const bool has_tau = (htau[3 * i] | htau[3 * i + 1] | htau[3 * i + 2]) != 0;
      if (has_tau && hk[i] > 0 && hge[i] < hk[i]) {
        htau[3 * i] = htau[3 * i + 1] = htau[3 * i + 2] = 0;
        redo = true;
      }
    }
    if (!redo) break;
    S.retries++;
    LP_HIP(hipMemcpyAsync(gtau, htau.data(), NG * 12, hipMemcpyHostToDevice, st));
  }
  S.appended = n_total;
  LP_HIP(hipEventRecord(tm.ev[2], st));
  // sort the buffer by (graph, score desc, a, c) and take each graph's first k
  LP_HIP(hipMemsetAsync(gcount, 0, (size_t)NG * 4, st));
  std::vector<uint32_t> hcount(NG);
  if (n_total > 0) {
    hipLaunchKernelGGL(graph_id_kernel, dim3(grid_for(n_total, 256, cus * 8)), dim3(256), 0, st, E.out_a,
                       n_total, gstart, NG, gid, gcount);
    LP_HIP(hipGetLastError());
    SortSpec sp{};
    sp.w[0] = gid;
    sp.w[1] = E.out_s;
    sp.w[2] = E.out_a;
    sp.w[3] = E.out_c;
    sp.nwords = 4;
    sp.nkeys = 4;
    sp.key_bits[0] = id_bits(NG);
    sp.key_bits[1] = 32;
    sp.key_bits[2] = id_bits((uint64_t)g->n);
    sp.key_bits[3] = id_bits((uint64_t)g->n);
    sp.invert[1] = true;
    LP_TRY(radix_sort(sp, (int64_t)n_total, w.sort_tmp, w.sort_counts, w.scan_tmp, st));
  }
  LP_TRY(scan_exclusive_u32(gcount, gseg, (int64_t)NG, w.scan_tmp, st));
  hipPointerAttribute_t at;
  const bool dev_out =
      hipPointerGetAttributes(&at, out_a) == hipSuccess && at.type == hipMemoryTypeDevice &&
      hipPointerGetAttributes(&at, out_c) == hipSuccess && at.type == hipMemoryTypeDevice &&
      hipPointerGetAttributes(&at, out_score) == hipSuccess && at.type == hipMemoryTypeDevice;
  (void)hipGetLastError();
  int32_t* xa = out_a;
  int32_t* xc = out_c;
  float* xs = out_score;
  if (!dev_out) {
    LP_TRY(w.q_out.ensure(ktot * 12 + 64));
    xa = w.q_out.as<int32_t>();
    xc = xa + ktot;
    xs = reinterpret_cast<float*>(xc + ktot);
  }
  if (n_total > 0) {
    hipLaunchKernelGGL(graph_take_kernel, dim3(grid_for(n_total, 256, cus * 8)), dim3(256), 0, st, gid,
                       E.out_s, E.out_a, E.out_c, n_total, gseg, gk, goff, xa, xc, xs);
    LP_HIP(hipGetLastError());
  }
  LP_HIP(hipMemcpyAsync(hcount.data(), gcount, NG * 4, hipMemcpyDeviceToHost, st));
  LP_HIP(hipEventRecord(tm.ev[3], st));
  LP_HIP(hipStreamSynchronize(st));
  if (!dev_out) {
    // each graph's rows sit at its output offset; copy only the filled ones
    for (uint32_t i = 0; i < NG; i++) {
      const uint64_t kout = std::min<uint64_t>(hk[i], hcount[i]);
      if (!kout) continue;
      LP_HIP(hipMemcpyAsync(out_a + hoff[i], xa + hoff[i], kout * 4, hipMemcpyDefault, st));
      LP_HIP(hipMemcpyAsync(out_c + hoff[i], xc + hoff[i], kout * 4, hipMemcpyDefault, st));
      LP_HIP(hipMemcpyAsync(out_score + hoff[i], xs + hoff[i], kout * 4, hipMemcpyDefault, st));
    }
    LP_HIP(hipStreamSynchronize(st));
  }
  uint32_t herr = 0;
  LP_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  if (herr) return set_error(LP_ERR_DEVICE, "device error flags 0x%x", herr);
  for (uint32_t i = 0; i < NG; i++) out_count[i] = (int64_t)std::min<uint64_t>(hk[i], hcount[i]);
  LP_TRY(collect_work(w, &S, st));
  S.ms_plan = tm.ms(0, 1);
  S.ms_accumulate = tm.ms(1, 2);
  S.ms_total = tm.ms(0, 3);
  S.ms_select = S.ms_total - S.ms_plan - S.ms_accumulate;
  return LP_OK;
}

lp_status run_fingerprint(lp_graph* g, int64_t L, uint64_t* out, hipStream_t st) {
  Workspace& w = g->ws;
  lp_stats& S = g->last;
  S = lp_stats{};
  PlanResult pr;
  LP_TRY(run_plan(g, L, &pr, st));
  S.wedges = pr.out.wedges;
  S.sources = pr.out.sources;
  for (int b = 0; b < kBuckets; b++) S.bucket_sources[b] = pr.out.count[b];
  uint32_t *ovf, *ovf_count, *err, *tau;
  void* ovf_rec;
  unsigned long long *count, *fp;
  uint32_t ovf_cap;
  LP_TRY(ensure_ovf(w, &ovf, &ovf_rec, &ovf_count, &ovf_cap, &err, &count, &fp, &tau, st));
  Emit E{};
  E.measure = LP_CN;
  E.shift = g->fixed_shift;
  E.s_th = 0;
  E.tau = tau;
  E.out_count = count;
  E.fp_mode = 1;
  E.fp = fp;
  E.ovf = ovf;
  E.ovf_rec = ovf_rec;
  E.ovf_count = ovf_count;
  E.ovf_cap = ovf_cap;
  E.err = err;
  uint32_t ovf_host = 0;
  if (pr.out.wedges) {
    LaunchClock clk(&S, w);
    LP_TRY(run_phase_any<false>(g, w, view_of(g), E, w.lists.as<SrcRec>(), (uint64_t)g->n,
                                pr.out.count, 1, 0, &ovf_host, &clk, st));
    LP_TRY(collect_work(w, &S, st));
  }
  unsigned long long h[3];
  uint32_t herr = 0;
  LP_HIP(hipMemcpyAsync(h, fp, 24, hipMemcpyDeviceToHost, st));
  LP_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  if (herr) return set_error(LP_ERR_DEVICE, "device error flags 0x%x", herr);
  out[0] = h[0];
  out[1] = h[1];
  out[2] = h[2];
  out[3] = pr.out.wedges;
  return LP_OK;
}

lp_status run_query(lp_graph* g, Workspace& w, const int32_t* sources, int64_t nq, int m, int64_t L,
                    int32_t kq, float s_th, int32_t* out_c, float* out_score, int32_t* out_count,
                    hipStream_t st) {
  if (nq == 0) return LP_OK;
  const uint64_t Q = (uint64_t)nq;
  // sources to device (validated on the host side by the caller)
  LP_TRY(w.q_src.ensure(Q * 4));
  LP_HIP(hipMemcpyAsync(w.q_src.p, sources, Q * 4, hipMemcpyDefault, st));
  // per query: a source record in the list of its bucket
  LP_TRY(w.q_rows.ensure(Q * sizeof(SrcRec) * kBuckets + 256));
  SrcRec* qlists = w.q_rows.as<SrcRec>();
  LP_TRY(w.stats.ensure(sizeof(PlanOut) + 64));
  LP_TRY(w.host_stats.ensure(kHostStatsBytes));
  PlanOut* d_out = w.stats.as<PlanOut>();
  LP_HIP(hipMemsetAsync(d_out, 0, sizeof(PlanOut), st));
  const uint32_t hub = hub_start(g, L);
  const AccConfig cfg = acc_config(g);
  const GView gv = view_of(g);
  hipLaunchKernelGGL(query_plan_kernel, dim3(grid_for(Q, 1, 65536)), dim3(256), 0, st, gv, hub,
                     cfg.cuts, w.q_src.as<int32_t>(), g->rank, (uint32_t)Q, qlists, d_out,
                     (const uint32_t*)nullptr);
  LP_HIP(hipGetLastError());
  PlanOut* hp = w.host_stats.as<PlanOut>();
  LP_HIP(hipMemcpyAsync(hp, d_out, sizeof(PlanOut), hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  const PlanOut po = *hp;
  if (po.bad_source) return set_error(LP_ERR_INVALID_ARGUMENT, "a source id is outside [0, n)");
  int wshift = 0;
  LP_TRY(weighted_shift(g, m, L, &wshift));
  uint64_t cap = std::max<uint64_t>(po.wedges, 1);
  if (cap > (1ull << 32) - 1) return set_error(LP_ERR_OUT_OF_MEMORY, "query batch too large");
  if (w.cand_s.fixed && cap * 4 > w.cand_s.cap)
    return set_error(LP_ERR_INVALID_ARGUMENT,
                     "the sources' two-hop path bound (%llu) exceeds the fixed scratch's candidate capacity (%zu)",
                     (unsigned long long)cap, w.cand_s.cap / 4);
  LP_TRY(w.cand_s.ensure(cap * 4));
  LP_TRY(w.cand_a.ensure(cap * 4));
  LP_TRY(w.cand_c.ensure(cap * 4));
  LP_TRY(w.q_cnt.ensure(Q * 8 + 64));
  uint32_t* seg_count = w.q_cnt.as<uint32_t>();
  uint32_t* seg_start = seg_count + Q;
  LP_HIP(hipMemsetAsync(seg_count, 0, Q * 4, st));
  uint32_t *ovf, *ovf_count, *err, *tau;
  void* ovf_rec;
  unsigned long long *count, *fp;
  uint32_t ovf_cap;
  LP_TRY(ensure_ovf(w, &ovf, &ovf_rec, &ovf_count, &ovf_cap, &err, &count, &fp, &tau, st));
  Emit E{};
  E.measure = m;
  E.shift = wshift;
  E.s_th = s_th;
  E.tau = tau;
  E.out_s = w.cand_s.as<uint32_t>();
  E.out_a = w.cand_a.as<uint32_t>();
  E.out_c = w.cand_c.as<uint32_t>();
  E.out_count = count;
  E.cap = cap;
  E.q_count = seg_count;
  E.kq = kq > 0 ? (uint32_t)kq : 0u;
  E.fp = fp;
  E.ovf = ovf;
  E.ovf_rec = ovf_rec;
  E.ovf_count = ovf_count;
  E.ovf_cap = ovf_cap;
  E.err = err;
  uint32_t ovf_host = 0;
  // lp_query (not a server slot) keeps the call's statistics
  const bool own_stats = &w == &g->ws;
  if (own_stats) g->last = lp_stats{};
  std::unique_ptr<LaunchClock> clk(own_stats ? new LaunchClock(&g->last, w) : nullptr);
  unsigned long long n_total = 0;
  Readback rb;
  rb.dst[0] = &n_total;
  rb.src[0] = count;
  rb.bytes[0] = 8;
  if (po.wedges)
    LP_TRY(run_phase_any<true>(g, w, gv, E, qlists, Q, po.count, 1, 0, &ovf_host, clk.get(), st, nullptr, &rb));
  if (n_total > cap) return set_error(LP_ERR_DEVICE, "query candidate overflow");
  if (own_stats) {
    LP_TRY(collect_work(w, &g->last, st));
    g->last.wedges = po.wedges;
    g->last.sources = po.sources;
    for (int b = 0; b < kBuckets; b++) g->last.bucket_sources[b] = po.count[b];
    g->last.appended = n_total;
  }
  // sort by (query index asc, score desc, c asc)
  if (n_total > 1) {
    SortSpec sp{};
    sp.w[0] = E.out_a;
    sp.w[1] = E.out_s;
    sp.w[2] = E.out_c;
    sp.nwords = 3;
    sp.nkeys = 3;
    sp.key_bits[0] = id_bits(Q);
    sp.key_bits[1] = 32;
    sp.key_bits[2] = id_bits((uint64_t)g->n);
    sp.invert[0] = false;
    sp.invert[1] = true;
    sp.invert[2] = false;
    LP_TRY(radix_sort(sp, (int64_t)n_total, w.sort_tmp, w.sort_counts, w.scan_tmp, st));
  }
  LP_TRY(scan_exclusive_u32(seg_count, seg_start, (int64_t)Q, w.scan_tmp, st));
  // outputs (device or host)
  hipPointerAttribute_t at;
  bool dev_out = hipPointerGetAttributes(&at, out_c) == hipSuccess && at.type == hipMemoryTypeDevice &&
                 hipPointerGetAttributes(&at, out_score) == hipSuccess && at.type == hipMemoryTypeDevice &&
                 hipPointerGetAttributes(&at, out_count) == hipSuccess && at.type == hipMemoryTypeDevice;
  (void)hipGetLastError();
  const uint64_t tot = Q * (uint64_t)kq;
  int32_t* dc = out_c;
  float* ds = out_score;
  int32_t* dn = out_count;
  if (!dev_out) {
    LP_TRY(w.sort_tmp[0].ensure(tot * 8 + Q * 4 + 64));
    dc = w.sort_tmp[0].as<int32_t>();
    ds = reinterpret_cast<float*>(dc + tot);
    dn = reinterpret_cast<int32_t*>(ds + tot);
  }
  hipLaunchKernelGGL(query_take_kernel, dim3(grid_for(tot, 256, 65536)), dim3(256), 0, st,
                     E.out_s, E.out_c, seg_start, seg_count, (uint32_t)Q, kq, dc, ds, dn,
                     (const uint32_t*)nullptr, (uint64_t)cap);
  LP_HIP(hipGetLastError());
  if (!dev_out) {
    LP_HIP(hipMemcpyAsync(out_c, dc, tot * 4, hipMemcpyDefault, st));
    LP_HIP(hipMemcpyAsync(out_score, ds, tot * 4, hipMemcpyDefault, st));
    LP_HIP(hipMemcpyAsync(out_count, dn, Q * 4, hipMemcpyDefault, st));
  }
  uint32_t herr = 0;
  LP_HIP(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st));
  LP_HIP(hipStreamSynchronize(st));
  if (herr) return set_error(LP_ERR_DEVICE, "device error flags 0x%x", herr);
  return LP_OK;
}

// ---------------------------------------------------------------------------
// The query path with every count on the device, for replay as a HIP graph:
// no host round trip, no allocation and no memset node between its first
// and last operation.  Sizes come from capacities fixed by the caller (the
// server's admission): at most qcap sources, a two-hop path bound (candidate
// capacity) of pcap, and `slabs` dense accumulators for sources above the LDS
// capacity and for overflowing tables (one workgroup each).  The host reads
// the call's status words afterwards; a batch whose candidates exceeded pcap
// or whose overflow list filled is run again by run_query.
// ---------------------------------------------------------------------------

namespace {

__global__ void zero_words_kernel(uint32_t* __restrict__ a, uint32_t na, uint32_t* __restrict__ b, uint32_t nb,
                                  uint32_t* __restrict__ c, uint32_t nc) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < na + nb + nc; i += stride) {
    if (i < na) a[i] = 0;
    else if (i < na + nb) b[i - na] = 0;
    else c[i - na - nb] = 0;
  }
}

// Scratch layout of the device query path (byte offsets into w.q_src and
// w.q_out; the pinned buffers mirror the first 64 bytes of each).
constexpr size_t kQHead = 64;     // q_src: the query count (u32), then the sources at kQHead
constexpr size_t kDqStatus = 512;  // host output: counters (256 B) and the plan record, then results

size_t dq_out_bytes(uint32_t qcap, int32_t kq) { return (size_t)qcap * kq * 8 + (size_t)qcap * 4; }

}  // namespace

// Layout of w.spa_meta for `slabs` sources per round: piece offsets of arcs
// and keys and the key counts (u32, slabs + 1 each), then per-source floors
// (u64) and sum histograms (u32, kSumBins each).
static size_t spa_meta_u32(unsigned slabs) { return ((size_t)slabs * 3 + 8 + 1) & ~(size_t)1; }
static size_t spa_meta_bytes(unsigned slabs) {
  return spa_meta_u32(slabs) * 4 + (size_t)slabs * 8 + (size_t)slabs * kSumBins * 4;
}

size_t query_device_in_bytes(uint32_t qcap) { return kQHead + (size_t)qcap * 4; }
size_t query_device_out_bytes(uint32_t qcap, int32_t kq) { return kDqStatus + dq_out_bytes(qcap, kq); }

uint64_t query_device_layout(const Workspace& w) {
  const void* p[16] = {w.q_src.p,      w.q_rows.p,      w.stats.p,       w.counters.p,    w.cand_s.p,
                       w.cand_a.p,     w.cand_c.p,      w.q_cnt.p,       w.global_tab.p,  w.sort_tmp[0].p,
                       w.sort_tmp[1].p, w.sort_tmp[2].p, w.sort_counts.p, w.scan_tmp.p,    w.q_out.p,
                       w.spa_meta.p};
  uint64_t h = 0x9E3779B97F4A7C15ull ^ w.global_slabs;
  for (const void* q : p) {
    h ^= (uint64_t)(uintptr_t)q;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 31;
  }
  return h;
}

lp_status query_device_reserve(lp_graph* g, Workspace& w, const QueryShape& sh, bool* moved, hipStream_t st) {
  const uint64_t before = query_device_layout(w);
  const uint64_t Q = sh.qcap;
  LP_TRY(w.q_src.ensure(query_device_in_bytes(sh.qcap)));
  LP_TRY(w.q_rows.ensure(Q * sizeof(SrcRec) * kBuckets + 256));
  LP_TRY(w.stats.ensure(sizeof(PlanOut) + 64));
  LP_TRY(w.counters.ensure(kCountersBytes));
  LP_TRY(w.cand_s.ensure(sh.pcap * 4));
  LP_TRY(w.cand_a.ensure(sh.pcap * 4));
  LP_TRY(w.cand_c.ensure(sh.pcap * 4));
  LP_TRY(w.q_cnt.ensure(Q * 8 + 64));
  const size_t n = (size_t)g->n;
  if (w.global_slabs < sh.slabs) {
    w.global_tab.release();
    w.global_slabs = 0;
    LP_TRY(w.global_tab.ensure((size_t)sh.slabs * n * 12));
    // accumulators start at zero and every workgroup leaves its slab so; the
    // clearing is ordered before the launches on the same stream (a
    // non-blocking stream does not wait for the null stream)
    LP_HIP(hipMemsetAsync(w.global_tab.p, 0, (size_t)sh.slabs * n * 8, st));
    w.global_slabs = sh.slabs;
  }
  LP_TRY(w.spa_meta.ensure(spa_meta_bytes(std::max(1u, w.global_slabs))));
  const int64_t ntiles = ((int64_t)sh.pcap + 2047) / 2048;
  for (int k = 0; k < 3; k++) LP_TRY(w.sort_tmp[k].ensure(sh.pcap * 4));
  LP_TRY(w.sort_counts.ensure((size_t)ntiles * 256 * 4 * 2));
  // the scans: sort counts (ntiles * 256 words) and the per-query counts
  const int64_t nscan = std::max<int64_t>(ntiles * 256, (int64_t)Q);
  LP_TRY(w.scan_tmp.ensure(scan_scratch_bytes(nscan)));
  LP_TRY(w.q_out.ensure(dq_out_bytes(sh.qcap, sh.kq) + 64));
  *moved = query_device_layout(w) != before;
  return LP_OK;
}

// `rounds` split rounds over the work list wl, sizes read on the device.
template <bool kW>
static lp_status split_rounds_device(lp_graph* g, Workspace& w, const GView& gv, const Emit& E, const WorkList& wl,
                                     unsigned slabs, unsigned rounds, hipStream_t st) {
  uint32_t* meta = w.spa_meta.as<uint32_t>();
  const size_t u32_meta = spa_meta_u32(slabs);
  unsigned long long* floor_sum = reinterpret_cast<unsigned long long*>(meta + u32_meta);
  uint32_t* hist = reinterpret_cast<uint32_t*>(floor_sum + slabs);
  const bool floors = kW && E.kq > 0;
  char* base = w.global_tab.as<char>();
  uint32_t* spa_keys = reinterpret_cast<uint32_t*>(base + (size_t)w.global_slabs * (size_t)g->n * 8);
  const unsigned grid = (unsigned)num_cus() * 4;
  for (unsigned r = 0; r < rounds; r++) {
    SpaRound R{wl,   r * slabs, slabs, meta, meta + slabs + 1, meta + 2 * (slabs + 1), base, spa_keys,
               hist, floors ? floor_sum : nullptr, wl.count_dev};
    const uint32_t nh = floors ? slabs * kSumBins : 0u;
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid_for((uint64_t)slabs + nh, 256, 1024)), dim3(256), 0, st,
                       R.nkeys, slabs, floors ? hist : nullptr, nh, (uint32_t*)nullptr, 0u);
    hipLaunchKernelGGL(spa_pieces_kernel, dim3(1), dim3(1024), 0, st, R, 0);
    hipLaunchKernelGGL((spa_split_acc_kernel<kW, true, false>), dim3(grid), dim3(kSpaThreads), 0, st, gv, E, R);
    hipLaunchKernelGGL((spa_split_excl_kernel<kW, true, false>), dim3(slabs), dim3(kSpaThreads), 0, st, gv, E, R);
    hipLaunchKernelGGL(spa_pieces_kernel, dim3(1), dim3(1024), 0, st, R, 1);
    if (floors) {
      hipLaunchKernelGGL((spa_split_hist_kernel<kW, true, false>), dim3(grid), dim3(kSpaThreads), 0, st, gv, E, R);
      hipLaunchKernelGGL(spa_split_floor_kernel, dim3(slabs), dim3(64), 0, st, R, E.kq);
    }
    hipLaunchKernelGGL((spa_split_sweep_kernel<kW, true, false>), dim3(grid), dim3(kSpaThreads), 0, st, gv, E, R);
    LP_HIP(hipGetLastError());
  }
  return LP_OK;
}

lp_status query_device_enqueue(lp_graph* g, Workspace& w, const QueryShape& sh, const void* host_in,
                               void* host_out, hipStream_t st) {
  const uint32_t Q = sh.qcap;
  const int32_t kq = sh.kq;
  // inputs: the query count and the sources, from pinned host memory
  LP_HIP(hipMemcpyAsync(w.q_src.p, host_in, query_device_in_bytes(Q), hipMemcpyHostToDevice, st));
  const uint32_t* nq_dev = w.q_src.as<uint32_t>();
  const int32_t* src = reinterpret_cast<const int32_t*>(w.q_src.as<char>() + kQHead);
  SrcRec* qlists = w.q_rows.as<SrcRec>();
  PlanOut* d_out = w.stats.as<PlanOut>();
  uint32_t* seg_count = w.q_cnt.as<uint32_t>();
  uint32_t* seg_start = seg_count + Q;
  uint32_t *ovf, *ovf_count, *err, *tau;
  void* ovf_rec;
  unsigned long long *count, *fp;
  uint32_t ovf_cap;
  ovf_layout(w, &ovf, &ovf_rec, &ovf_count, &ovf_cap, &err, &count, &fp, &tau);
  hipLaunchKernelGGL(zero_words_kernel, dim3(grid_for((uint64_t)Q + 2048, 256, 1024)), dim3(256), 0, st,
                     reinterpret_cast<uint32_t*>(d_out), (uint32_t)(sizeof(PlanOut) / 4), seg_count, Q,
                     w.counters.as<uint32_t>(), 1024u);
  LP_HIP(hipGetLastError());
  const uint32_t hub = hub_start(g, sh.L);
  const AccConfig cfg = acc_config(g);
  const GView gv = view_of(g);
  hipLaunchKernelGGL(query_plan_kernel, dim3(grid_for(Q, 1, 65536)), dim3(256), 0, st, gv, hub, cfg.cuts, src,
                     g->rank, Q, qlists, d_out, nq_dev);
  LP_HIP(hipGetLastError());
  Emit E{};
  E.measure = sh.m;
  LP_TRY(weighted_shift(g, sh.m, sh.L, &E.shift));
  E.s_th = sh.s_th;
  E.tau = tau;
  E.out_s = w.cand_s.as<uint32_t>();
  E.out_a = w.cand_a.as<uint32_t>();
  E.out_c = w.cand_c.as<uint32_t>();
  E.out_count = count;
  E.cap = sh.pcap;
  E.q_count = seg_count;
  E.kq = (uint32_t)kq;
  E.fp = fp;
  E.ovf = ovf;
  E.ovf_rec = ovf_rec;
  E.ovf_count = ovf_count;
  E.ovf_cap = ovf_cap;
  E.err = err;
  unsigned long long* work = work_counters(w);
  const bool kw = sh.m == LP_AA || sh.m == LP_RA;
  char* base = w.global_tab.as<char>();
  uint32_t* spa_keys = reinterpret_cast<uint32_t*>(base + (size_t)w.global_slabs * (size_t)g->n * 8);
  const unsigned slabs = std::max(1u, w.global_slabs);
  for (int b = kBuckets - 1; b >= 0; b--) {
    WorkList wl{qlists + (uint64_t)b * Q, 0, 1, 0, &d_out->count[b]};
    E.work = work + b * 8;
    if (b == kBucketHuge) {
      // sources above the LDS capacity: rounds of one dense slab each, every
      // source split over all CUs (as the host-driven path does for a few);
      // a shape with no rounds has none of them
      if (sh.rounds == 0) continue;
      if (kw) LP_TRY(split_rounds_device<true>(g, w, gv, E, wl, slabs, sh.rounds, st));
      else LP_TRY(split_rounds_device<false>(g, w, gv, E, wl, slabs, sh.rounds, st));
    } else if (kw) {
      LP_TRY((launch_bucket_tables<kTabSplit, true, false>(g, b, gv, E, wl, Q, st)));
    } else {
      LP_TRY((launch_bucket_tables<kTabCount, true, false>(g, b, gv, E, wl, Q, st)));
    }
  }
  // partitions of sources whose LDS table filled up, on the dense accumulators
  E.work = work + kBucketHuge * 8;
  {
    const WorkList none{nullptr, 0, 1, 0};
    const SpaItem ov{ovf, static_cast<const SrcRec*>(ovf_rec), 0, ovf_cap, ovf_count};
    if (kw)
      hipLaunchKernelGGL((acc_spa_kernel<true, true, false>), dim3(slabs), dim3(kSpaThreads), 0, st, gv, E, none,
                         ov, base, spa_keys);
    else
      hipLaunchKernelGGL((acc_spa_kernel<false, true, false>), dim3(slabs), dim3(kSpaThreads), 0, st, gv, E,
                         none, ov, base, spa_keys);
    LP_HIP(hipGetLastError());
  }
  // by (query index asc, score desc, c asc), over the candidates counted on the device
  SortSpec sp{};
  sp.w[0] = E.out_a;
  sp.w[1] = E.out_s;
  sp.w[2] = E.out_c;
  sp.nwords = 3;
  sp.nkeys = 3;
  sp.key_bits[0] = id_bits(Q);
  sp.key_bits[1] = 32;
  sp.key_bits[2] = id_bits((uint64_t)g->n);
  sp.invert[0] = false;
  sp.invert[1] = true;
  sp.invert[2] = false;
  uint32_t* where[4];
  LP_TRY(radix_sort_device_count(sp, (int64_t)sh.pcap, count, w.sort_tmp, w.sort_counts, w.scan_tmp, st, where));
  LP_TRY(scan_exclusive_u32(seg_count, seg_start, (int64_t)Q, w.scan_tmp, st));
  const uint64_t tot = (uint64_t)Q * (uint64_t)kq;
  int32_t* dc = w.q_out.as<int32_t>();
  float* ds = reinterpret_cast<float*>(dc + tot);
  int32_t* dn = reinterpret_cast<int32_t*>(ds + tot);
  hipLaunchKernelGGL(query_take_kernel, dim3(grid_for(tot, 256, 65536)), dim3(256), 0, st, where[1], where[2],
                     seg_start, seg_count, Q, kq, dc, ds, dn, nq_dev, (uint64_t)sh.pcap);
  LP_HIP(hipGetLastError());
  // status words (counters block: candidate count, overflow count, error
  // flags) and the plan's record, then the results
  char* ho = static_cast<char*>(host_out);
  LP_HIP(hipMemcpyAsync(ho, w.counters.p, 256, hipMemcpyDeviceToHost, st));
  LP_HIP(hipMemcpyAsync(ho + 256, d_out, sizeof(PlanOut), hipMemcpyDeviceToHost, st));
  LP_HIP(hipMemcpyAsync(ho + kDqStatus, dc, dq_out_bytes(Q, kq), hipMemcpyDeviceToHost, st));
  return LP_OK;
}

lp_status query_device_status(const void* host_out, const QueryShape& sh, uint32_t nq,
                              uint64_t* candidates) {
  const char* ho = static_cast<const char*>(host_out);
  unsigned long long n_total;
  uint32_t ovf_total, herr;
  PlanOut po;
  std::memcpy(&n_total, ho, 8);
  std::memcpy(&ovf_total, ho + 128, 4);
  std::memcpy(&herr, ho + 192, 4);
  std::memcpy(&po, ho + 256, sizeof(PlanOut));
  if (candidates) *candidates = n_total;
  if (po.bad_source) return set_error(LP_ERR_INVALID_ARGUMENT, "a source id is outside [0, n)");
  if (herr) return set_error(LP_ERR_DEVICE, "device error flags 0x%x", herr);
  (void)nq;
  // beyond the capacities of the replayed launches: the caller runs the
  // batch again on the host-driven path
  if (n_total > sh.pcap || ovf_total > kOvfCap || po.count[kBucketHuge] > (uint64_t)sh.rounds * sh.slabs)
    return LP_ERR_OUT_OF_MEMORY;
  return LP_OK;
}

}  // namespace lp

// kernels.h - device building blocks of the two-hop accumulation, fused
// scoring and candidate emission.  Included by predict.hip only.
#pragma once

#include "lp_common.h"

namespace lp {

constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr uint32_t kHashMul = 0x9E3779B1u;            // Fibonacci hashing multiplier

// Read-only view of the resident graph (relabelled ids).
struct GView {
  const uint32_t* off;
  const uint32_t* adj;
  const uint32_t* hoff;    // two-hop arc list (arcs with wedges c > a)
  const uint32_t* hdeg;    // degree of each arc's intermediate
  const uint32_t* hstart;
  const uint32_t* hpsum;
  const uint32_t* deg;
  const uint32_t* below;
  const uint32_t* perm;
  const uint32_t* deg_first;  // [deg_cap + 1] first id whose degree is >= d
  uint32_t deg_cap;
  uint32_t n;
};

// Where and how candidates leave the scoring epilogue.
struct Emit {
  int measure;
  int shift;               // fixed-point fraction bits of AA / RA sums
  float s_th;              // keep FP32 scores strictly above this
  const uint32_t* tau;     // [3] key threshold (score bits, ~a, ~c); keep key >= tau
  uint32_t* out_s;         // score bits
  uint32_t* out_a;         // predict: smaller original id; query: query index
  uint32_t* out_c;         // predict: larger original id; query: original id of c
  unsigned long long* out_count;
  unsigned long long cap;
  uint32_t* q_count;       // query: candidates per query index (may be null)
  int fp_mode;             // accumulate the candidate-set digest instead of emitting
  unsigned long long* fp;  // [3] digest accumulators
  uint32_t* ovf;           // overflow records: (pass | P << 8) per entry
  void* ovf_rec;           // overflow records: the source record per entry
  uint32_t* ovf_count;
  uint32_t ovf_cap;
  uint32_t* err;           // error flags
  unsigned long long* work;  // [5] this launch's work counters (lp_bucket_stats order)
  // several graphs at once: graph i owns original ids [gstart[i], gstart[i+1])
  // and keeps keys >= gtau[3i..3i+2]; null gtau: tau applies to every source
  const uint32_t* gtau;
  const uint32_t* gstart;
  uint32_t ngraphs;
  uint32_t kq;  // query: results wanted per source (0: keep every candidate)
  // packed AA / RA tables (key and fixed-point sum in one 64-bit slot): id
  // bits of a key (0: 12-byte tables); a source whose sums do not fit is
  // listed in unfit_rec and accumulated afterwards with 12-byte tables
  int pk_idbits;
  void* unfit_rec;  // SrcRec[unfit_cap]
  uint32_t* unfit_count;
  uint32_t unfit_cap;
};


// Log-scale bins of a positive fixed-point sum: values below 8 have a bin
// each, then eight bins per octave (bin order = value order), 496 in all.
constexpr uint32_t kSumBins = 512;
__device__ inline uint32_t sum_bin(uint64_t v) {
  if (v < 8) return (uint32_t)v;
  const uint32_t o = 63u - (uint32_t)__clzll((long long)v);  // octave, >= 3
  return 8u + (o - 3u) * 8u + (uint32_t)((v >> (o - 3u)) & 7u);
}
// smallest sum in bin b
__device__ inline uint64_t sum_bin_floor(uint32_t b) {
  if (b < 8) return b;
  const uint32_t o = (b - 8u) / 8u + 3u, sub = (b - 8u) % 8u;
  return (uint64_t)(8u + sub) << (o - 3u);
}

// Graph of an original id (several-graph calls only).
__device__ inline uint32_t graph_of(const Emit& E, uint32_t key) {
  uint32_t lo = 0, hi = E.ngraphs;  // gstart[lo] <= key < gstart[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (E.gstart[mid] <= key) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Threshold key of the source with original id key (predict orientation).
__device__ inline const uint32_t* tau_of(const Emit& E, uint32_t key) {
  return E.gtau ? E.gtau + 3 * graph_of(E, key) : E.tau;
}

// Work counters of one lane (sources, sum d_a, arcs, wedges, candidates),
// added to the launch's totals once per wave at the end of a kernel.
struct WorkAcc {
  unsigned long long v[5] = {0, 0, 0, 0, 0};
  __device__ void source(uint32_t da, uint32_t na, uint32_t U) {
    v[0] += 1;
    v[1] += da;
    v[2] += na;
    v[3] += U;
  }
};

__device__ inline void flush_work(const Emit& E, WorkAcc& wa) {
#pragma unroll
  for (int i = 0; i < 5; i++) {
    unsigned long long x = wa.v[i];
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(&E.work[i], x);
  }
}

enum : uint32_t { kErrProbe = 1, kErrOvfList = 2 };

// Hand a whole source to the 12-byte-table launch that follows a packed
// phase (or, without one, to the global path as an overflow record).
template <class Rec>
__device__ inline void hand_unfit(const Emit& E, const Rec& r) {
  if (E.unfit_rec) {
    const uint32_t slot = atomicAdd(E.unfit_count, 1u);
    if (slot < E.unfit_cap) static_cast<Rec*>(E.unfit_rec)[slot] = r;
    else atomicOr(E.err, kErrOvfList);
    return;
  }
  const uint32_t slot = atomicAdd(E.ovf_count, 1u);
  if (slot < E.ovf_cap) {
    static_cast<Rec*>(E.ovf_rec)[slot] = r;
    E.ovf[slot] = 0u | (1u << 8);
  } else {
    atomicOr(E.err, kErrOvfList);
  }
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ inline uint64_t mix64(uint64_t a, uint64_t c, uint64_t h) {
  uint64_t z = ((a << 32) | (c & 0xFFFFFFFFull)) ^ (h * 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline bool needs_dc(int m) { return m >= LP_JC && m <= LP_LHN; }

// Section 3.1 measures, evaluated in FP64 (AA / RA from the fixed-point sum).
__device__ inline double score_of(int m, uint32_t h, uint64_t wsum, uint32_t da, uint32_t dc,
                                  int shift) {
  const double H = (double)h;
  switch (m) {
    case LP_CN: return H;
    case LP_JC: return H / (double)((uint64_t)da + dc - h);
    case LP_SI: return H / (double)((uint64_t)da + dc);
    case LP_SC: return H / sqrt((double)da * (double)dc);
    case LP_HP: return H / (double)(da < dc ? da : dc);
    case LP_HD: return H / (double)(da > dc ? da : dc);
    case LP_LHN: return H / ((double)da * (double)dc);
    default: return ldexp((double)wsum, -shift);
  }
}

// fixed-point weight of an explored intermediate of degree db
__device__ inline uint64_t weight_of(int m, uint32_t db, int shift) {
  if (m == LP_AA) return db > 1 ? (uint64_t)llrint(ldexp(1.0 / log((double)db), shift)) : 0ull;
  return db > 0 ? (uint64_t)llrint(ldexp(1.0 / (double)db, shift)) : 0ull;
}

// Upper bounds of each measure that need only h and d_a (h <= d_a always;
// d_c >= h always, and d_c >= d_a when the candidate follows the source in the
// degree order, "ordered"):
//   ordered:   JC <= h / (2 d_a - h), SI <= h / (2 d_a), SC, HP, HD <= h / d_a,
//              LHN <= h / d_a^2
//   unordered: JC, HD <= h / d_a, SI <= h / (d_a + h), SC <= sqrt(h / d_a),
//              LHN <= 1 / d_a, HP <= 1
// CN is h itself.  Rounding to FP32 is monotone, so the FP32 value of a bound
// bounds the FP32 score.
__device__ inline float bound_score(int m, uint32_t h, uint32_t da, bool ordered) {
  const double H = (double)h, A = (double)da;
  if (ordered) {
    switch (m) {
      case LP_CN: return (float)H;
      case LP_JC: return (float)(H / (2.0 * A - H));
      case LP_SI: return (float)(H / (2.0 * A));
      case LP_SC:
      case LP_HP:
      case LP_HD: return (float)(H / A);
      case LP_LHN: return (float)(H / (A * A));
      default: return 3.0e38f;
    }
  }
  switch (m) {
    case LP_CN: return (float)H;
    case LP_JC:
    case LP_HD: return (float)(H / A);
    case LP_SI: return (float)(H / (A + H));
    case LP_SC: return (float)(H / sqrt(A * H));
    case LP_LHN: return (float)(H / (A * H));
    default: return 3.0e38f;
  }
}

// Smallest count h a candidate of a source of degree da needs for its FP32
// score to reach the threshold score ts; 0xFFFFFFFF when no candidate of the
// source can reach it.  AA / RA use min_wsum instead.
__device__ inline uint32_t min_count(int m, uint32_t ts_bits, uint32_t da, bool ordered) {
  if (ts_bits == 0 || m == LP_AA || m == LP_RA || (m == LP_HP && !ordered)) return 1u;
  const float ts = __uint_as_float(ts_bits);
  const uint32_t hmax = da < 0xFFFFFFu ? da : 0xFFFFFFu;  // h <= d_a; counts stay below 2^24
  if (hmax == 0 || bound_score(m, hmax, da, ordered) < ts) return 0xFFFFFFFFu;
  // closed-form estimate of the crossing, then exact correction steps
  const double t = (double)ts, A = (double)da;
  double est;
  switch (m) {
    case LP_CN: est = t; break;
    case LP_JC: est = ordered ? 2.0 * t * A / (1.0 + t) : t * A; break;
    case LP_SI: est = ordered ? 2.0 * t * A : (t < 1.0 ? t * A / (1.0 - t) : A); break;
    case LP_SC: est = ordered ? t * A : t * t * A; break;
    case LP_LHN: est = ordered ? t * A * A : 1.0; break;
    default: est = t * A; break;  // HP, HD
  }
  uint32_t h = est < 1.0 ? 1u : (est > (double)hmax ? hmax : (uint32_t)est);
  while (h < hmax && bound_score(m, h, da, ordered) < ts) h++;
  while (h > 1 && bound_score(m, h - 1, da, ordered) >= ts) h--;
  return h;
}

// Candidates with count h of a source of degree da can reach the score lo
// only if d_c stays below a bound that follows from the measure:
//   JC: d_c <= h / lo + h - d_a   SI: d_c <= h / lo - d_a
//   SC: d_c <= h^2 / (lo^2 d_a)   LHN: d_c <= h / (lo d_a)
//   HD: d_c <= h / lo (ordered: d_c >= d_a)
// Ids are in degree order, so that is an id cutoff: candidates with an id
// at or above the returned value cannot pass (0xFFFFFFFF: no cutoff).  The
// bound is rounded up, so no passing candidate is ever cut.
__device__ inline uint32_t id_cutoff(int m, uint32_t h, uint32_t da, double lo, const GView& g,
                                     bool ordered) {
  if (!(lo > 0.0) || da == 0) return 0xFFFFFFFFu;
  const double H = (double)h, A = (double)da;
  double X;
  switch (m) {
    case LP_JC: X = H / lo + H - A; break;
    case LP_SI: X = H / lo - A; break;
    case LP_SC: X = H * H / (lo * lo * A); break;
    case LP_HD:
      if (!ordered) return 0xFFFFFFFFu;
      X = H / lo;
      break;
    case LP_LHN: X = H / (lo * A); break;
    default: return 0xFFFFFFFFu;
  }
  X = X * (1.0 + 0x1p-40) + 1e-6;
  if (!(X < (double)g.deg_cap)) return 0xFFFFFFFFu;
  if (X < 0.0) return 0u;
  return g.deg_first[(uint32_t)X + 1];
}

// Lower edge of the exact scores whose FP32 value can pass the threshold key
// (score >= ts) and the score threshold (score > s_th): the midpoint between
// ts and the float below it, or s_th when that is higher.
__device__ inline double pass_edge(uint32_t ts_bits, float s_th) {
  double lo = (double)s_th;
  if (ts_bits != 0) {
    const double mid = 0.5 * ((double)__uint_as_float(ts_bits - 1u) + (double)__uint_as_float(ts_bits));
    lo = mid > lo ? mid : lo;
  }
  return lo;
}

// True when the exact score is certainly below lo, tested as h < lo * d (d
// the measure's denominator) without dividing; the right-hand side is taken
// 2^-50 low so that its rounding can never reject a score >= lo.
__device__ inline bool score_below(int m, uint32_t h, uint64_t wsum, uint32_t da, uint32_t dc,
                                   int shift, double lo) {
  constexpr double kLow = 1.0 - 0x1p-50;
  const double H = (double)h;
  switch (m) {
    case LP_CN: return H < lo;
    case LP_JC: return H < lo * (double)((uint64_t)da + dc - h) * kLow;
    case LP_SI: return H < lo * (double)((uint64_t)da + dc) * kLow;
    case LP_SC: return H * H < lo * lo * (double)da * (double)dc * kLow;
    case LP_HP: return H < lo * (double)(da < dc ? da : dc) * kLow;
    case LP_HD: return H < lo * (double)(da > dc ? da : dc) * kLow;
    case LP_LHN: return H < lo * (double)da * (double)dc * kLow;
    default: return ldexp((double)wsum, -shift) < lo * kLow;
  }
}

// AA / RA: a fixed-point sum below this cannot reach ts (conservative: sums
// under the FP32 value just below ts round to at most that value)
__device__ inline uint64_t min_wsum(int m, uint32_t ts_bits, int shift) {
  if (ts_bits <= 1u || (m != LP_AA && m != LP_RA)) return 1ull;
  const double below = (double)__uint_as_float(ts_bits - 1u);  // positive floats: bits are ordered
  const double est = floor(ldexp(below, shift));
  if (!(est < 1.8e19)) return ~0ull;  // no fixed-point sum reaches it
  return est < 1.0 ? 1ull : (uint64_t)est;
}


struct FpAcc {
  unsigned long long cnt = 0, sh = 0, sm = 0;
};

// Per-wave staging in LDS, two levels.  The table sweep stages candidate
// entries (c, h or weight sum, source) that pass the source's count bound;
// their degree / id loads, FP64 scoring and threshold test run in batches
// (stage_score), off the per-source dependency chain.  Survivors go to a
// second stage that reaches global memory with one device-scope atomic per
// batch (stage_out).  All stage calls are made by every lane of a wave at the
// same point, so the fill counts live in wave-uniform registers.
struct Stage {
  uint32_t* c;   // [cap] candidate (relabelled id)
  uint32_t* h;   // [cap] count, or low word of the AA / RA sum
  uint32_t* w2;  // [cap] high word of the AA / RA sum (weighted tables only)
  uint32_t* k;   // [cap] predict: source's original id; query: query index
  uint32_t* d;   // [cap] source degree
  uint32_t cap;
  uint32_t* os;  // [ocap] survivors: score bits
  uint32_t* oa;  // [ocap] survivors: smaller original id / query index
  uint32_t* oc;  // [ocap] survivors: larger original id / original id of c
  uint32_t ocap;
  uint32_t n = 0;   // candidates held
  uint32_t on = 0;  // survivors held
};

__device__ inline void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }
// The floor of the highest bin that completes k_q sums, from one wave over a
// kSumBins histogram (0 when there are fewer than k_q sums: keep all).
// Lane l reads bins [8 l, 8 l + 8); the result is wave-uniform.
__device__ inline uint64_t sum_floor_wave(const uint32_t* h, uint32_t kq) {
  const int lane = lane_id();
  const uint32_t* mine = h + lane * 8;
  uint32_t sum = 0;
  for (int i = 0; i < 8; i++) sum += mine[i];
  // entries in the lanes above (suffix sums over lanes)
  uint32_t above = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_down(above, o, 64);
    if (lane + o < 64) above += y;
  }
  above -= sum;
  // the bin that completes k_q: at most one lane has it
  uint32_t bin = 0xFFFFFFFFu;
  if (above < kq && above + sum >= kq) {
    uint32_t run = above;
    for (int i = 7; i >= 0 && bin == 0xFFFFFFFFu; i--) {
      run += mine[i];
      if (run >= kq) bin = (uint32_t)(lane * 8 + i);
    }
  }
  // wave minimum of the candidate bins (0xFFFFFFFF: fewer than k_q sums)
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t y = __shfl_xor(bin, o, 64);
    bin = y < bin ? y : bin;
  }
  return bin == 0xFFFFFFFFu ? 0ull : sum_bin_floor(bin);
}

__device__ inline uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t uniform64(uint64_t v) {
  return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// Copy the survivors to the global buffer.
template <bool kQuery>
__device__ inline void stage_out(const Emit& E, Stage& S) {
  if (S.on == 0) return;
  wave_fence();
  unsigned long long base = 0;
  if (lane_id() == 0) base = atomicAdd(E.out_count, (unsigned long long)S.on);
  base = __shfl(base, 0);
  for (uint32_t j = lane_id(); j < S.on; j += 64) {
    const unsigned long long pos = base + j;
    const uint32_t a = S.oa[j];
    if (pos < E.cap) {
      E.out_s[pos] = S.os[j];
      E.out_a[pos] = a;
      E.out_c[pos] = S.oc[j];
    }
    if (kQuery && E.q_count) atomicAdd(&E.q_count[a], 1u);
  }
  wave_fence();
  S.on = 0;
}

// Score the staged candidates; survivors move to the survivor stage.
template <bool kQuery, bool kW>
__device__ inline void stage_score(const Emit& E, const GView& g, Stage& S, FpAcc& fa) {
  if (S.n == 0) return;
  wave_fence();
  const bool want_dc = needs_dc(E.measure);
  uint32_t t0 = E.tau[0], t1 = E.tau[1], t2 = E.tau[2];
  double lo = pass_edge(E.fp_mode ? 0u : t0, E.s_th);
  for (uint32_t j0 = 0; j0 < S.n; j0 += 64) {
    const uint32_t j = j0 + lane_id();
    const bool in = j < S.n;
    const uint32_t jc = in ? j : 0u;
    const uint32_t c = S.c[jc], h = S.h[jc], k = S.k[jc], da = S.d[jc];
    if (!kQuery && E.gtau) {  // each source keeps its own graph's threshold
      const uint32_t* t = tau_of(E, k);
      t0 = t[0];
      t1 = t[1];
      t2 = t[2];
      lo = pass_edge(t0, E.s_th);
    }
    const uint64_t wsum = kW ? (((uint64_t)S.w2[jc] << 32) | h) : 0ull;
    const uint32_t dc = want_dc ? g.deg[c] : 0u;
    // most staged candidates fail the threshold: reject those without
    // dividing and without loading the original id
    bool live = in;
    if (!E.fp_mode) live = live & !score_below(E.measure, h, wsum, da, dc, E.shift, lo);
    uint32_t co = 0, sb = 0;
    float f = 0.0f;
    if (live) {
      co = g.perm[c];
      f = (float)score_of(E.measure, h, wsum, da, dc, E.shift);
      sb = __float_as_uint(f);
    }
    const uint32_t ka = kQuery ? k : (k < co ? k : co);
    const uint32_t kc = kQuery ? co : (k < co ? co : k);
    bool keep = false;
    if (E.fp_mode) {
      if (in) {
        fa.cnt += 1;
        fa.sh += h;
        fa.sm += mix64(ka, kc, h);
      }
    } else if (live && f > E.s_th) {
      if (kQuery) keep = sb > t0 || (sb == t0 && (~kc) >= t2);
      else keep = sb > t0 || (sb == t0 && ((~ka) > t1 || ((~ka) == t1 && (~kc) >= t2)));
    }
    const uint64_t m = __ballot(keep);
    const uint32_t nk = (uint32_t)__popcll(m);
    if (nk == 0) continue;
    if (S.on + nk > S.ocap) stage_out<kQuery>(E, S);
    if (keep) {
      const uint32_t p = S.on + (uint32_t)__popcll(m & lanemask_lt());
      S.os[p] = sb;
      S.oa[p] = ka;
      S.oc[p] = kc;
    }
    S.on += nk;
  }
  wave_fence();
  S.n = 0;
}

// Stage the valid lanes' entries (all lanes of the wave call this together).
template <bool kQuery, bool kW>
__device__ inline void stage_add(const Emit& E, const GView& g, Stage& S, bool valid, uint32_t c,
                                 uint32_t h, uint64_t wsum, uint32_t key, uint32_t da, FpAcc& fa) {
  const uint64_t m = __ballot(valid);
  const uint32_t nk = (uint32_t)__popcll(m);
  if (nk == 0) return;
  if (S.n + nk > S.cap) stage_score<kQuery, kW>(E, g, S, fa);
  if (valid) {
    const uint32_t j = S.n + (uint32_t)__popcll(m & lanemask_lt());
    S.c[j] = c;
    S.h[j] = kW ? (uint32_t)wsum : h;
    if (kW) S.w2[j] = (uint32_t)(wsum >> 32);
    S.k[j] = key;
    S.d[j] = da;
  }
  S.n += nk;
}

// Drain both stages (end of a kernel).
template <bool kQuery, bool kW>
__device__ inline void stage_drain(const Emit& E, const GView& g, Stage& S, FpAcc& fa) {
  stage_score<kQuery, kW>(E, g, S, fa);
  if (!E.fp_mode) stage_out<kQuery>(E, S);
}

// ---------------------------------------------------------------------------
// Open-addressing tables in LDS (linear probing, S slots, keys < 2^31).
// Every probe loop runs a uniform trip count over the wave; each lane works
// on K keys at once so that K independent LDS round trips are in flight.
//   count table:    one 64-bit slot per key, (count << 32) | key
//   weighted table: keys[S] (32-bit) and vals[S] (64-bit fixed-point sums)
// A first-order neighbour's entry is flagged with kBlocked in its count or
// kBlocked64W in its sum, and dropped when the table is swept.
// ---------------------------------------------------------------------------

constexpr uint32_t kBlocked = 0x80000000u;
constexpr uint64_t kSlotEmpty = 0x00000000FFFFFFFFull;  // key empty, count 0
constexpr uint64_t kSlotOne = 1ull << 32;               // count increment
constexpr uint64_t kBlocked64 = (uint64_t)kBlocked << 32;
constexpr uint64_t kBlocked64W = 1ull << 63;

__device__ inline uint32_t next_slot(uint32_t h, uint32_t S) { return h + 1 == S ? 0u : h + 1; }

// popcount(M & lanes below this one), in two instructions
__device__ inline uint32_t rank_lt(uint64_t M) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(M >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)M, 0u));
}

// Table updates carry a 64-bit increment: for count tables kSlotOne (a wedge)
// or kBlocked64 (the key is a first-order neighbour of the source), for
// weighted tables the fixed-point weight of the wedge's intermediate or
// kBlocked64W.  A key is blocked at most once and sums stay below 2^62, so
// adding the flag sets it.  The sweep drops flagged entries.

// Probe from slot h on until key lands (key == kEmpty32: nothing to do);
// the loop runs until every lane of the wave is done.  False if the table is
// full for some lane.
__device__ inline bool probe_count(uint64_t* tab, uint32_t S, uint32_t key, uint32_t h, uint64_t inc) {
  for (uint32_t probe = 0; probe < S; probe++) {
    if (!__any(key != kEmpty32)) return true;
    uint64_t old = kSlotEmpty;
    if (key != kEmpty32)
      old = atomicCAS((unsigned long long*)&tab[h], (unsigned long long)kSlotEmpty,
                      (unsigned long long)(inc | key));
    // lanes without a live key saw old == kSlotEmpty and stay dead
    const bool same = (key != kEmpty32) & ((uint32_t)old == key);
    if (same) atomicAdd((unsigned long long*)&tab[h], (unsigned long long)inc);
    key = (same | (old == kSlotEmpty)) ? kEmpty32 : key;
    h = next_slot(h, S);
  }
  return !__any(key != kEmpty32);
}

__device__ inline bool probe_weight(uint32_t* keys, uint64_t* vals, uint32_t S, uint32_t key, uint32_t h,
                                    uint64_t inc) {
  for (uint32_t probe = 0; probe < S; probe++) {
    if (!__any(key != kEmpty32)) return true;
    uint32_t old = 0;
    if (key != kEmpty32) old = atomicCAS(&keys[h], kEmpty32, key);
    const bool hit = (key != kEmpty32) & ((old == kEmpty32) | (old == key));
    if (hit) atomicAdd((unsigned long long*)&vals[h], (unsigned long long)inc);
    key = hit ? kEmpty32 : key;
    h = next_slot(h, S);
  }
  return !__any(key != kEmpty32);
}

// Packed weighted table (AA / RA in prediction orientation): one 64-bit slot
// per key, bit 63 the first-order flag, bits [kb, 63) a fixed-point sum with a
// per-source number of fraction bits, bits [0, kb) the key; an empty slot
// holds the key mask kmask = 2^kb - 1 (no key reaches it).  A new key costs
// one compare-and-swap, like a count table (which is this layout with kb = 32
// and a sum that counts wedges).
__device__ inline bool probe_packed(uint64_t* tab, uint32_t S, uint32_t key, uint32_t h, uint64_t inc,
                                    uint32_t kmask) {
  const uint64_t empty = kmask;
  for (uint32_t probe = 0; probe < S; probe++) {
    if (!__any(key != kEmpty32)) return true;
    uint64_t old = empty;
    if (key != kEmpty32)
      old = atomicCAS((unsigned long long*)&tab[h], (unsigned long long)empty,
                      (unsigned long long)(inc | key));
    // lanes without a live key saw old == empty and stay dead
    const bool same = (key != kEmpty32) & (((uint32_t)old & kmask) == key);
    if (same) atomicAdd((unsigned long long*)&tab[h], (unsigned long long)inc);
    key = (same | (old == empty)) ? kEmpty32 : key;
    h = next_slot(h, S);
  }
  return !__any(key != kEmpty32);
}

// Table modes of the LDS accumulation kernels.
enum : int {
  kTabCount = 0,   // (count << 32) | key per 64-bit slot
  kTabSplit = 1,   // weighted: 32-bit keys and 64-bit fixed-point sums (12 bytes per slot)
  kTabPacked = 2   // weighted: key and fixed-point sum in one 64-bit slot
};

// Per-wave list of insertions whose home slot held another key.  Every key
// gets one probe where it falls; the few that need more wait here and are
// probed on in batches of up to 64, so that one long probe sequence does not
// hold up the 63 other lanes of its window.  Used by all lanes of a wave
// together; the fill count is wave-uniform.  Count tables keep the kind of
// increment in bit 31 of the slot index (set: blocked).
template <bool kW>
struct Retry {
  uint32_t* key;  // [64]
  uint32_t* h;    // [64] next slot to probe
  uint64_t* w;    // [64] increment (weighted tables only)
  uint32_t n = 0;
};

template <int TM>
__device__ inline bool retry_drain(uint64_t* tab, uint32_t* keys, uint64_t* vals, uint32_t S,
                                   Retry<TM != kTabCount>& R, uint32_t kmask = kEmpty32) {
  constexpr bool kW = TM != kTabCount;
  if (R.n == 0) return true;
  wave_fence();
  const uint32_t l = (uint32_t)lane_id();
  const bool in = l < R.n;
  const uint32_t key = in ? R.key[l] : kEmpty32;
  const uint32_t hv = in ? R.h[l] : 0u;
  const uint64_t w = (kW && in) ? R.w[l] : 0ull;
  wave_fence();
  R.n = 0;
  if (TM == kTabSplit) return probe_weight(keys, vals, S, key, hv, w);
  if (TM == kTabPacked) return probe_packed(tab, S, key, hv, w, kmask);
  return probe_count(tab, S, key, hv & ~kBlocked, (hv & kBlocked) ? kBlocked64 : kSlotOne);
}

// Add inc to key's entry, inserting the key if absent (key == kEmpty32: no
// update on this lane).  False if the table is full for some key.  kmask:
// key mask of a packed table.
template <int TM>
__device__ inline bool tab_insert(uint64_t* tab, uint32_t* keys, uint64_t* vals, uint32_t S, uint32_t key,
                                  uint32_t h, uint64_t inc, Retry<TM != kTabCount>& R,
                                  uint32_t kmask = kEmpty32) {
  const bool live = key != kEmpty32;
  bool done;
  if (TM == kTabSplit) {
    uint32_t old = 0;
    if (live) old = atomicCAS(&keys[h], kEmpty32, key);
    done = (old == kEmpty32) | (old == key);
    if (live & done) atomicAdd((unsigned long long*)&vals[h], (unsigned long long)inc);
  } else if (TM == kTabPacked) {
    const uint64_t empty = kmask;
    uint64_t old = empty;
    if (live)
      old = atomicCAS((unsigned long long*)&tab[h], (unsigned long long)empty,
                      (unsigned long long)(inc | key));
    const bool same = live & (((uint32_t)old & kmask) == key);
    if (same) atomicAdd((unsigned long long*)&tab[h], (unsigned long long)inc);
    done = same | (old == empty);
  } else {
    uint64_t old = kSlotEmpty;
    if (live)
      old = atomicCAS((unsigned long long*)&tab[h], (unsigned long long)kSlotEmpty,
                      (unsigned long long)(inc | key));
    const bool same = (uint32_t)old == key;
    if (live & same) atomicAdd((unsigned long long*)&tab[h], (unsigned long long)inc);
    done = same | (old == kSlotEmpty);
  }
  const bool fail = live & !done;
  const uint64_t M = __ballot(fail);
  if (M == 0) return true;
  const uint32_t nf = (uint32_t)__popcll(M);
  bool ok = true;
  if (R.n + nf > 64) ok = retry_drain<TM>(tab, keys, vals, S, R, kmask);
  if (fail) {
    const uint32_t p = R.n + rank_lt(M);
    R.key[p] = key;
    const uint32_t hn = next_slot(h, S);
    if (TM != kTabCount) {
      R.h[p] = hn;
      R.w[p] = inc;
    } else {
      R.h[p] = inc == kSlotOne ? hn : (hn | kBlocked);
    }
  }
  R.n += nf;
  return ok;
}

// Key c's home slot in a table of S slots (a mix of the bits, then range
// reduction to [0, S)).
__device__ inline uint32_t key_slot(uint32_t c, uint32_t S) {
  const uint32_t x = (c ^ (c >> 15)) * 0x2C1B3C6Du;
  return (uint32_t)(((uint64_t)(x ^ (x >> 12)) * S) >> 32);
}

// K keys per lane at once into a count or packed table: every
// compare-and-swap is issued before any result is used, so the K LDS round
// trips overlap; then hits add their increments and misses join the retry
// list.  Adds commute and a compare-and-swap looks only at the key bits, so
// the order of the K updates does not matter.  key[u] == kEmpty32: none.
template <int TM, int K>
__device__ inline bool tab_insert_k(uint64_t* tab, uint32_t S, const uint32_t (&key)[K],
                                    const uint64_t (&inc)[K], Retry<TM != kTabCount>& R, uint32_t kmask) {
  static_assert(TM != kTabSplit, "one 64-bit slot per key");
  const uint64_t empty = TM == kTabPacked ? (uint64_t)kmask : kSlotEmpty;
  const uint32_t km = TM == kTabPacked ? kmask : 0xFFFFFFFFu;
  uint32_t h[K];
  uint64_t old[K];
#pragma unroll
  for (int u = 0; u < K; u++) {
    h[u] = key_slot(key[u], S);
    old[u] = empty;
    if (key[u] != kEmpty32)
      old[u] = atomicCAS((unsigned long long*)&tab[h[u]], (unsigned long long)empty,
                         (unsigned long long)(inc[u] | key[u]));
  }
  bool ok = true;
#pragma unroll
  for (int u = 0; u < K; u++) {
    const bool live = key[u] != kEmpty32;
    const bool same = live & (((uint32_t)old[u] & km) == key[u]);
    if (same) atomicAdd((unsigned long long*)&tab[h[u]], (unsigned long long)inc[u]);
    const bool fail = live & !same & (old[u] != empty);
    const uint64_t M = __ballot(fail);
    if (M == 0) continue;
    const uint32_t nf = (uint32_t)__popcll(M);
    if (R.n + nf > 64) ok = retry_drain<TM>(tab, nullptr, nullptr, S, R, kmask) & ok;
    if (fail) {
      const uint32_t p = R.n + rank_lt(M);
      R.key[p] = key[u];
      const uint32_t hn = next_slot(h[u], S);
      if (TM == kTabPacked) {
        R.h[p] = hn;
        R.w[p] = inc[u];
      } else {
        R.h[p] = inc[u] == kSlotOne ? hn : (hn | kBlocked);
      }
    }
    R.n += nf;
  }
  return ok;
}

// Whether a source's packed sums fit: a key's sum has at most na terms (one
// per explored arc), each below 2^e (RA: 1/d_b <= 1/2, e = -1; AA: 1/ln d_b
// <= 1/ln 2 < 2, e = 1); with F fraction bits and each term rounded to
// nearest, the sum stays below 2^(ceil(log2 na) + e + F + 1), which must fit
// the 63 - kb bits above the key.
__device__ inline bool packed_fits(int m, uint32_t na, int kb, int F) {
  const int lg = na <= 1 ? 0 : 32 - __clz((int)(na - 1));  // ceil(log2 na)
  return lg + (m == LP_RA ? -1 : 1) + F + 1 <= 63 - kb;
}

// The fixed-point sum of a packed slot.
__device__ inline uint64_t packed_sum(uint64_t v, int kb) { return (v << 1) >> (kb + 1); }

// ---------------------------------------------------------------------------
// Run-length decoding of a chunk of arcs into wedges, one wave at a time.
// Arc j of the chunk covers the flat wedge offsets [excl[j], excl[j + 1]);
// arcs are never empty.  A wave walks windows of 64 consecutive offsets; lane
// p takes offset base + p.  j is the (wave-uniform) arc that holds base on
// entry and base + 64 on exit; mark is a per-wave array of 64 bytes that is
// zero between calls.  Returns the lane's arc.
// ---------------------------------------------------------------------------

__device__ inline uint32_t decode_window(const uint32_t* excl, uint32_t narcs, uint8_t* mark,
                                         uint32_t base, uint32_t& j) {
  const uint32_t lane = (uint32_t)lane_id();
  const uint32_t t = j + 1 + lane;
  if (t < narcs) {
    const uint32_t pos = excl[t] - base;  // >= 1: arc j holds base
    if (pos < 64) mark[pos] = 1;
  }
  wave_fence();
  const bool m = mark[lane] != 0;
  mark[lane] = 0;
  wave_fence();
  const uint64_t M = __ballot(m);
  const uint32_t arc = j + rank_lt(M) + (m ? 1u : 0u);
  j = uniform(j + (uint32_t)__popcll(M));
  return arc;
}

__device__ inline void flush_fp(const Emit& E, FpAcc& fa) {
  if (!E.fp_mode) return;
  unsigned long long c = fa.cnt, h = fa.sh, s = fa.sm;
  for (int o = 32; o >= 1; o >>= 1) {
    c += __shfl_xor(c, o);
    h += __shfl_xor(h, o);
    s += __shfl_xor(s, o);
  }
  if (lane_id() == 0 && (c | h)) {
    atomicAdd(&E.fp[0], c);
    atomicAdd(&E.fp[1], h);
    atomicAdd(&E.fp[2], s);
  }
}

// Synchronisation of the lanes that share one table.
template <int G>
__device__ inline void group_sync() {
  if constexpr (G > 64) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}

// Exclusive prefix sum of one value per lane within a group of G lanes
// (G <= 64: shuffles inside the wave; G > 64: through LDS).
template <int G>
__device__ inline uint32_t group_exclusive_scan(uint32_t v, uint32_t* lds_tmp /*[G / 64]*/,
                                                uint32_t* total) {
  const int gl = threadIdx.x & (G - 1);
  if constexpr (G <= 64) {
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      uint32_t y = __shfl_up(x, o, G);
      if (gl >= o) x += y;
    }
    *total = __shfl(x, G - 1, G);
    return x - v;
  } else {
    const int l = lane_id(), w = gl >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t y = __shfl_up(x, o, 64);
      if (l >= o) x += y;
    }
    if (l == 63) lds_tmp[w] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < G / 64; i++) {
      if (i < w) base += lds_tmp[i];
      tot += lds_tmp[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
  }
}

// index of the last entry <= f in a non-decreasing array of G entries whose
// first entry is <= f
template <int G>
__device__ inline int seg_search(const uint32_t* s, uint32_t f) {
  int lo = 0;
#pragma unroll
  for (int step = G / 2; step >= 1; step >>= 1)
    if (s[lo + step] <= f) lo += step;
  return lo;
}

}  // namespace lp

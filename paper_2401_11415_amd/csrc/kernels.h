// kernels.h - device building blocks of the two-hop accumulation, fused
// scoring and candidate emission.  Included by predict.hip only.
#pragma once

#include "lp_common.h"

namespace lp {

constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr uint64_t kEmpty64 = 0xFFFFFFFF00000000ull;  // key = empty, count = 0
constexpr uint32_t kHashMul = 0x9E3779B1u;            // Fibonacci hashing multiplier

// Read-only view of the resident graph (relabelled ids).
struct GView {
  const uint32_t* off;
  const uint32_t* adj;
  const uint32_t* hoff;    // two-hop arc list (arcs with wedges c > a)
  const uint32_t* hb;
  const uint32_t* hstart;
  const uint32_t* hpsum;
  const uint32_t* deg;
  const uint32_t* below;
  const uint32_t* perm;
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
  uint32_t* ovf;           // overflow records (source, pass | lgP << 8)
  uint32_t* ovf_count;
  uint32_t ovf_cap;
  uint32_t* err;           // error flags
};

enum : uint32_t { kErrProbe = 1, kErrOvfList = 2 };

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

struct FpAcc {
  unsigned long long cnt = 0, sh = 0, sm = 0;
};

// Per-wave staging of surviving candidates in LDS: survivors are collected
// here and copied to the global buffer with one atomic per flush, instead of
// one device-scope atomic per (wave, sweep step) with any survivor.
struct Stage {
  uint32_t* s;    // [cap] score bits
  uint32_t* a;    // [cap]
  uint32_t* c;    // [cap]
  uint32_t* cnt;  // entries held (one LDS word per wave)
  uint32_t cap;
};

// The staged count is shared by the lanes of a wave through LDS: atomic
// accesses keep the compiler from reusing a lane's own stale copy.
__device__ inline uint32_t stage_count(const Stage& S) {
  return __hip_atomic_load(S.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ inline void stage_set_count(const Stage& S, uint32_t v) {
  __hip_atomic_store(S.cnt, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Copy the staged entries out; callable with any set of active lanes.
__device__ inline void stage_flush(const Emit& E, const Stage& S) {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const uint32_t n = stage_count(S);
  if (n == 0) return;
  const uint64_t act = __ballot(true);
  const int leader = __ffsll((unsigned long long)act) - 1;
  const uint32_t nact = (uint32_t)__popcll(act);
  const uint32_t ar = (uint32_t)__popcll(act & lanemask_lt());
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(E.out_count, (unsigned long long)n);
  base = __shfl(base, leader);
  for (uint32_t j = ar; j < n; j += nact) {
    const unsigned long long pos = base + j;
    if (pos < E.cap) {
      E.out_s[pos] = S.s[j];
      E.out_a[pos] = S.a[j];
      E.out_c[pos] = S.c[j];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  if (lane_id() == leader) stage_set_count(S, 0u);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// Score one (source, c) entry and stage it if it survives S_th and tau.
// Must be called by every active lane of the wave at the same point (ranks
// come from a ballot); lanes with valid == false pass through.
//   kQuery: a_key = query index, the pair is (source, c) ordered by c only.
//   dc: degree of c (needed by the normalised measures), loaded by the caller.
template <bool kQuery>
__device__ inline void emit_one(const Emit& E, const GView& g, const Stage& S, bool valid,
                                uint32_t a_orig, uint32_t a_key, uint32_t da, uint32_t c,
                                uint32_t dc, uint32_t h, uint64_t wsum, FpAcc& fa) {
  bool keep = false;
  uint32_t sb = 0, ka = 0, kc = 0;
  bool have_ids = false;
  if (valid) {
    const double s = score_of(E.measure, h, wsum, da, dc, E.shift);
    const float f = (float)s;
    sb = __float_as_uint(f);
    if (E.fp_mode) {
      const uint32_t co = g.perm[c];
      const uint32_t lo = a_orig < co ? a_orig : co, hi = a_orig < co ? co : a_orig;
      fa.cnt += 1;
      fa.sh += h;
      fa.sm += mix64(lo, hi, h);
    } else {
      keep = f > E.s_th;
      if (keep) {
        const uint32_t ts = E.tau[0];
        if (sb < ts) {
          keep = false;
        } else if (sb == ts) {
          const uint32_t co = g.perm[c];
          if (kQuery) {
            ka = a_key;
            kc = co;
            keep = (~kc) >= E.tau[2];
          } else {
            ka = a_orig < co ? a_orig : co;
            kc = a_orig < co ? co : a_orig;
            const uint32_t na = ~ka, nc = ~kc;
            keep = na > E.tau[1] || (na == E.tau[1] && nc >= E.tau[2]);
          }
          have_ids = true;
        }
      }
    }
  }
  if (E.fp_mode) return;
  const uint64_t m = __ballot(keep);
  if (m == 0) return;
  const uint32_t nk = (uint32_t)__popcll(m);
  if (stage_count(S) + nk > S.cap) stage_flush(E, S);
  const uint32_t base = stage_count(S);
  if (keep) {
    if (!have_ids) {
      const uint32_t co = g.perm[c];
      if (kQuery) {
        ka = a_key;
        kc = co;
      } else {
        ka = a_orig < co ? a_orig : co;
        kc = a_orig < co ? co : a_orig;
      }
    }
    const uint32_t j = base + (uint32_t)__popcll(m & lanemask_lt());
    S.s[j] = sb;
    S.a[j] = ka;
    S.c[j] = kc;
    if (kQuery && E.q_count) atomicAdd(&E.q_count[a_key], 1u);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  if (lane_id() == __ffsll((unsigned long long)m) - 1) stage_set_count(S, base + nk);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
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

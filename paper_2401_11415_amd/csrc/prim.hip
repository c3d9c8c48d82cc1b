// prim.hip - device scans and a stable LSD radix sort (gfx950, wave64).
#include <cstdarg>
#include <cstdio>

#include "lp_common.h"

namespace lp {

// ---------------------------------------------------------------------------
// Errors and buffers
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

lp_status set_error(lp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

void clear_error() { g_last_error.clear(); }

lp_status from_hip(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return set_error(LP_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
  return set_error(LP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error_text() { return g_last_error.c_str(); }

thread_local size_t ScratchLimit::bytes = 0;

lp_status DevBuf::ensure(size_t bytes) {
  if (bytes <= cap && p) return LP_OK;
  if (fixed)
    return set_error(LP_ERR_INVALID_ARGUMENT, "needs %zu bytes of a fixed scratch buffer of %zu bytes",
                     bytes, cap);
  size_t want = bytes ? bytes : 256;
  if (ScratchLimit::bytes && want > ScratchLimit::bytes)
    return set_error(LP_ERR_OUT_OF_MEMORY, "scratch allocation of %zu bytes above the limit of %zu",
                     want, ScratchLimit::bytes);
  release();
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return from_hip(e, "hipMalloc");
  }
  cap = want;
  return LP_OK;
}

void DevBuf::release() {
  if (fixed) return;
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
}

lp_status HostBuf::ensure(size_t bytes) {
  if (bytes <= cap && p) return LP_OK;
  if (fixed)
    return set_error(LP_ERR_INVALID_ARGUMENT, "needs %zu bytes of a fixed host staging buffer of %zu bytes",
                     bytes, cap);
  release();
  size_t want = bytes ? bytes : 256;
  hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return from_hip(e, "hipHostMalloc");
  }
  cap = want;
  return LP_OK;
}

void HostBuf::release() {
  if (fixed) return;
  if (p) (void)hipHostFree(p);
  p = nullptr;
  cap = 0;
}

int num_cus() {
  static int cached = 0;
  if (!cached) {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cu > 0)
      cached = cu;
    else
      cached = 256;
  }
  return cached;
}

size_t device_memory() {
  static size_t cached = 0;
  if (!cached) {
    size_t free_b = 0, total_b = 0;
    cached = hipMemGetInfo(&free_b, &total_b) == hipSuccess && total_b > 0 ? total_b : (size_t)64 << 30;
  }
  return cached;
}

// ---------------------------------------------------------------------------
// Block scan helpers (256 threads = 4 waves of 64)
// ---------------------------------------------------------------------------

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ inline T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// exclusive scan of one value per thread across the block; *total receives the sum
template <class T>
__device__ inline T block_exclusive_scan(T v, T* lds4, T* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = wave_inclusive_scan(v);
  if (lane == 63) lds4[wid] = x;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; w++) {
    if (w < wid) base += lds4[w];
    tot += lds4[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

template <class Tin, class Tacc>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const Tin* __restrict__ in,
                                                                   Tacc* __restrict__ sums,
                                                                   int64_t n) {
  __shared__ Tacc lds4[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  Tacc s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++)
    if (base + j < n) s += (Tacc)in[base + j];
  Tacc tot;
  (void)block_exclusive_scan<Tacc>(s, lds4, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[i] = offset + prefix (exclusive or inclusive) within the block
template <class Tin, class Tout, bool kInclusive>
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const Tin* __restrict__ in,
                                                                  Tout* __restrict__ out,
                                                                  const Tout* __restrict__ block_base,
                                                                  int64_t n) {
  __shared__ Tout lds4[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  Tout v[kScanItems];
  Tout s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    v[j] = (base + j < n) ? (Tout)in[base + j] : (Tout)0;
    s += v[j];
  }
  Tout tot;
  Tout run = block_exclusive_scan<Tout>(s, lds4, &tot);
  if (block_base) run += block_base[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    if (kInclusive) run += v[j];
    if (base + j < n) out[base + j] = run;
    if (!kInclusive) run += v[j];
  }
}

template <class Tin, class Tout, bool kInclusive>
static lp_status scan_impl(const Tin* in, Tout* out, int64_t n, DevBuf& tmp, hipStream_t st,
                           size_t tmp_off) {
  if (n <= 0) return LP_OK;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL((scan_apply_kernel<Tin, Tout, kInclusive>), dim3(1), dim3(kScanThreads), 0,
                       st, in, out, (const Tout*)nullptr, n);
    LP_HIP(hipGetLastError());
    return LP_OK;
  }
  // block sums live in tmp at tmp_off; their exclusive scan in place
  size_t need = tmp_off + (size_t)nb * sizeof(Tout) * 2 + 4096;
  if (tmp.cap < need) {
    return set_error(LP_ERR_OUT_OF_MEMORY, "scan scratch too small (%zu < %zu)", tmp.cap, need);
  }
  Tout* sums = reinterpret_cast<Tout*>(static_cast<char*>(tmp.p) + tmp_off);
  Tout* sums_scan = sums + nb;
  hipLaunchKernelGGL((scan_reduce_kernel<Tin, Tout>), dim3((unsigned)nb), dim3(kScanThreads), 0, st,
                     in, sums, n);
  LP_HIP(hipGetLastError());
  size_t next_off = tmp_off + (size_t)nb * sizeof(Tout) * 2;
  next_off = (next_off + 255) & ~(size_t)255;
  LP_TRY((scan_impl<Tout, Tout, false>(sums, sums_scan, nb, tmp, st, next_off)));
  hipLaunchKernelGGL((scan_apply_kernel<Tin, Tout, kInclusive>), dim3((unsigned)nb),
                     dim3(kScanThreads), 0, st, in, out, (const Tout*)sums_scan, n);
  LP_HIP(hipGetLastError());
  return LP_OK;
}

static size_t scan_tmp_bytes(int64_t n, size_t elem) {
  size_t total = 4096;
  int64_t m = n;
  while (m > kScanTile) {
    int64_t nb = (m + kScanTile - 1) / kScanTile;
    total += (size_t)nb * elem * 2 + 256;
    m = nb;
  }
  return total;
}

size_t scan_scratch_bytes(int64_t n) { return scan_tmp_bytes(n, sizeof(uint64_t)); }

lp_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, DevBuf& tmp,
                             hipStream_t st) {
  LP_TRY(tmp.ensure(scan_tmp_bytes(n, sizeof(uint32_t))));
  return scan_impl<uint32_t, uint32_t, false>(in, out, n, tmp, st, 0);
}

lp_status scan_inclusive_u32_u64(const uint32_t* in, uint64_t* out, int64_t n, DevBuf& tmp,
                                 hipStream_t st) {
  LP_TRY(tmp.ensure(scan_tmp_bytes(n, sizeof(uint64_t))));
  return scan_impl<uint32_t, uint64_t, true>(in, out, n, tmp, st, 0);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort: 8-bit digits, tiles of 2048 records per workgroup
// (the scatter stages a tile in LDS, 8 KB per record word, so small tiles
// let five workgroups share a CU for three-word records).
// Pass = per-tile digit histogram -> digit-major exclusive scan -> stable
// scatter through LDS.
// ---------------------------------------------------------------------------

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;

struct PassArgs {
  const uint32_t* in[4];
  uint32_t* out[4];
  int nwords;
  int key_word;
  int shift;
  uint32_t invert;                 // all-ones to complement the key word
  const unsigned long long* n_dev;  // if set: the record count, read on the device (at most n)
};

__device__ inline int64_t records_of(const PassArgs& p, int64_t n) {
  if (!p.n_dev) return n;
  const unsigned long long d = *p.n_dev;
  return d < (unsigned long long)n ? (int64_t)d : n;
}

__device__ inline uint32_t digit_of(const PassArgs& p, int64_t i) {
  uint32_t k = p.in[p.key_word][i] ^ p.invert;
  return (k >> p.shift) & 255u;
}

// Per-tile digit histogram.  Lanes add into kCountCopies histograms by lane
// number (rows padded to spread them over the LDS banks), so a run of equal
// digits (equal scores are common) serialises over 64 / kCountCopies lanes
// instead of the whole wave.
constexpr int kCountCopies = 16;

__global__ __launch_bounds__(kSortThreads) void radix_count_kernel(PassArgs p, int64_t n,
                                                                   uint32_t* __restrict__ counts,
                                                                   int64_t ntiles) {
  __shared__ uint32_t hist[kCountCopies][257];
  n = records_of(p, n);
  for (int j = 0; j < kCountCopies; j++) hist[j][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  uint32_t* mine = hist[threadIdx.x % kCountCopies];
#pragma unroll 4
  for (int r = 0; r < kSortItems; r++) {
    int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&mine[digit_of(p, i)], 1u);
  }
  __syncthreads();
  uint32_t tot = 0;
#pragma unroll
  for (int j = 0; j < kCountCopies; j++) tot += hist[j][threadIdx.x];
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = tot;
}

// Stable scatter of one tile: every wave ranks its quarter of the tile by digit
// (ballot match per round of 64, running per-digit counts in LDS), the tile
// is staged in LDS in digit order, and the staged records leave in runs of
// equal digits, so that neighbouring lanes write neighbouring addresses.
template <int NW>
struct ScatterLds {
  uint32_t words[NW][kSortTile];
  uint8_t dig[kSortTile];
  uint32_t wcnt[kSortThreads / 64][256];  // per-wave digit counts, then per-wave digit starts
  uint32_t dstart[256];                    // tile-local start of each digit
  uint32_t gbase[256];                     // global start of each digit for this tile
  uint32_t lds4[4];
};

template <int NW>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(PassArgs p, int64_t n,
                                                                     const uint32_t* __restrict__ offs,
                                                                     int64_t ntiles) {
  __shared__ ScatterLds<NW> L;
  constexpr int kWaves = kSortThreads / 64;
  constexpr int kRounds = kSortTile / kWaves / 64;  // rounds of 64 records per wave
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  n = records_of(p, n);
  for (int w = 0; w < kWaves; w++) L.wcnt[w][threadIdx.x] = 0;
  L.gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  __syncthreads();
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const int tile_n = (int)(n - tile0 < kSortTile ? n - tile0 : kSortTile);
  uint32_t item[kRounds][NW];
  uint32_t dg[kRounds], loc[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; r++) {
    const int t = (wid * kRounds + r) * 64 + lane;
    const bool valid = t < tile_n;
    uint32_t d = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) item[r][k] = valid ? p.in[k][tile0 + t] : 0u;
    uint32_t key = item[r][0];  // select the key word without indexing registers
#pragma unroll
    for (int k = 1; k < NW; k++) key = p.key_word == k ? item[r][k] : key;
    if (valid) d = ((key ^ p.invert) >> p.shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    // every lane reads its digit's running count before the leader (the
    // lowest lane with that digit) advances it
    const uint32_t base = L.wcnt[wid][d];
    if (valid && (m & lt) == 0) L.wcnt[wid][d] = base + (uint32_t)__popcll(m);
    dg[r] = d;
    loc[r] = base + (uint32_t)__popcll(m & lt);
  }
  __syncthreads();
  // digit totals -> tile-local digit starts -> per-wave starts
  uint32_t tot = 0;
  for (int w = 0; w < kWaves; w++) tot += L.wcnt[w][threadIdx.x];
  uint32_t all;
  const uint32_t ds = block_exclusive_scan<uint32_t>(tot, L.lds4, &all);
  L.dstart[threadIdx.x] = ds;
  uint32_t run = ds;
  for (int w = 0; w < kWaves; w++) {
    const uint32_t c = L.wcnt[w][threadIdx.x];
    L.wcnt[w][threadIdx.x] = run;
    run += c;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; r++) {
    const int t = (wid * kRounds + r) * 64 + lane;
    if (t < tile_n) {
      const uint32_t pos = L.wcnt[wid][dg[r]] + loc[r];
#pragma unroll
      for (int k = 0; k < NW; k++) L.words[k][pos] = item[r][k];
      L.dig[pos] = (uint8_t)dg[r];
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < tile_n; q += kSortThreads) {
    const uint32_t d = L.dig[q];
    const uint32_t dst = L.gbase[d] + ((uint32_t)q - L.dstart[d]);
#pragma unroll
    for (int k = 0; k < NW; k++) p.out[k][dst] = L.words[k][q];
  }
}

// n: the record count, or with n_dev its upper bound (the count itself is
// read on the device, so no host round trip is needed).  Sorted records end
// in spec.w, or with where != nullptr wherever the last pass left them
// (where[k] receives word k's buffer).
static lp_status radix_sort_impl(const SortSpec& spec, int64_t n, const unsigned long long* n_dev,
                                 DevBuf tmp[4], DevBuf& counts, DevBuf& scan_tmp, hipStream_t st,
                                 uint32_t** where) {
  if (n <= 1) {
    if (where)
      for (int k = 0; k < 4; k++) where[k] = spec.w[k];
    return LP_OK;
  }
  if (n >= (int64_t)UINT32_MAX) return set_error(LP_ERR_INVALID_ARGUMENT, "sort too large");
  const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
  for (int k = 0; k < spec.nwords; k++) LP_TRY(tmp[k].ensure((size_t)n * 4));
  LP_TRY(counts.ensure((size_t)ntiles * 256 * 4 * 2));
  uint32_t* cnts = counts.as<uint32_t>();
  uint32_t* offs = cnts + ntiles * 256;
  uint32_t* cur[4] = {spec.w[0], spec.w[1], spec.w[2], spec.w[3]};
  uint32_t* alt[4] = {tmp[0].as<uint32_t>(), tmp[1].as<uint32_t>(), tmp[2].as<uint32_t>(),
                      tmp[3].as<uint32_t>()};
  int passes = 0;
  for (int kw = spec.nkeys - 1; kw >= 0; kw--) {
    for (int shift = 0; shift < spec.key_bits[kw]; shift += 8) {
      PassArgs pa{};
      for (int k = 0; k < 4; k++) {
        pa.in[k] = cur[k];
        pa.out[k] = alt[k];
      }
      pa.nwords = spec.nwords;
      pa.key_word = kw;
      pa.shift = shift;
      pa.invert = spec.invert[kw] ? 0xFFFFFFFFu : 0u;
      pa.n_dev = n_dev;
      hipLaunchKernelGGL(radix_count_kernel, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, pa,
                         n, cnts, ntiles);
      LP_HIP(hipGetLastError());
      LP_TRY(scan_exclusive_u32(cnts, offs, ntiles * 256, scan_tmp, st));
      switch (spec.nwords) {
        case 1:
          hipLaunchKernelGGL(radix_scatter_kernel<1>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, pa, n,
                             (const uint32_t*)offs, ntiles);
          break;
        case 2:
          hipLaunchKernelGGL(radix_scatter_kernel<2>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, pa, n,
                             (const uint32_t*)offs, ntiles);
          break;
        case 3:
          hipLaunchKernelGGL(radix_scatter_kernel<3>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, pa, n,
                             (const uint32_t*)offs, ntiles);
          break;
        default:
          hipLaunchKernelGGL(radix_scatter_kernel<4>, dim3((unsigned)ntiles), dim3(kSortThreads), 0, st, pa, n,
                             (const uint32_t*)offs, ntiles);
          break;
      }
      LP_HIP(hipGetLastError());
      for (int k = 0; k < 4; k++) {
        uint32_t* t = cur[k];
        cur[k] = alt[k];
        alt[k] = t;
      }
      passes++;
    }
  }
  if (where) {
    for (int k = 0; k < 4; k++) where[k] = cur[k];
  } else if (passes & 1) {
    for (int k = 0; k < spec.nwords; k++)
      LP_HIP(hipMemcpyAsync(spec.w[k], cur[k], (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  }
  return LP_OK;
}

lp_status radix_sort(const SortSpec& spec, int64_t n, DevBuf tmp[4], DevBuf& counts,
                     DevBuf& scan_tmp, hipStream_t st) {
  return radix_sort_impl(spec, n, nullptr, tmp, counts, scan_tmp, st, nullptr);
}

lp_status radix_sort_device_count(const SortSpec& spec, int64_t n_cap, const unsigned long long* n_dev,
                                  DevBuf tmp[4], DevBuf& counts, DevBuf& scan_tmp, hipStream_t st,
                                  uint32_t** where) {
  return radix_sort_impl(spec, n_cap, n_dev, tmp, counts, scan_tmp, st, where);
}

}  // namespace lp

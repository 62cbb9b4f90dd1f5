// Stable LSD radix sort of (key, u32 value) pairs on the device: the sort of
// visible Gaussians by depth and of (tile, Gaussian) pairs by tile that put
// every tile's list in front-to-back (depth, index) order.
//
// Per 8-bit digit pass: (1) per-block digit histogram, (2) exclusive scan of
// the digit-major histogram table, (3) stable scatter.  Inside a block the
// rank of a key among equal digits comes from wave64 match masks: eight
// ballots give each lane the set of lanes holding its digit, the popcount of
// that set below the lane is its rank, and one leader lane per digit updates
// the running count.  No atomics, so the order is deterministic and stable.
#include "lgs_internal.h"

namespace lgs {
namespace {

constexpr int kThreads = 256;           // 4 waves
constexpr int kIters = 16;              // 64-key rows per wave
constexpr int kWaveKeys = 64 * kIters;  // 1024
constexpr int kTile = 4 * kWaveKeys;    // 4096 keys per block

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
  return (uint32_t)(k >> shift) & 255u;
}

__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
  uint64_t peers = valid;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __builtin_amdgcn_ballot_w64(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

__device__ __forceinline__ int64_t count_of(const uint32_t* n_dev, int64_t n_max) {
  return n_dev ? (int64_t)*n_dev : n_max;
}

template <typename K>
__global__ void __launch_bounds__(kThreads) k_hist(const K* __restrict__ keys, const uint32_t* n_dev,
                                                   int64_t n_max, int shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[4][256];
  const int64_t n = count_of(n_dev, n_max);
  const int64_t nb = (n + kTile - 1) / kTile;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (base >= n) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < 4 * 256; d += kThreads) (&cnt[0][0])[d] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int it = 0; it < kIters; ++it) {
    const int64_t i = base + wave * kWaveKeys + it * 64 + lane;
    const bool ok = i < n;
    const uint32_t d = ok ? digit_of(keys[i], shift) : 0u;
    const uint64_t valid = __builtin_amdgcn_ballot_w64(ok);
    const uint64_t peers = match_digit(d, valid);
    if (ok && (peers & lt) == 0ull) cnt[wave][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  const int d = threadIdx.x;
  hist[(int64_t)d * nb + blockIdx.x] = cnt[0][d] + cnt[1][d] + cnt[2][d] + cnt[3][d];
}

template <typename K>
__global__ void __launch_bounds__(kThreads) k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                      K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                      const uint32_t* n_dev, int64_t n_max, int shift,
                                                      const uint32_t* __restrict__ off) {
  __shared__ uint32_t cnt[4][256];
  const int64_t n = count_of(n_dev, n_max);
  const int64_t nb = (n + kTile - 1) / kTile;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (base >= n) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < 4 * 256; d += kThreads) (&cnt[0][0])[d] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  K kk[kIters];
  uint32_t vv[kIters];
  for (int it = 0; it < kIters; ++it) {
    const int64_t i = base + wave * kWaveKeys + it * 64 + lane;
    const bool ok = i < n;
    kk[it] = ok ? kin[i] : (K)0;
    vv[it] = ok ? vin[i] : 0u;
    const uint32_t d = digit_of(kk[it], shift);
    const uint64_t valid = __builtin_amdgcn_ballot_w64(ok);
    const uint64_t peers = match_digit(d, valid);
    if (ok && (peers & lt) == 0ull) cnt[wave][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t run = off[(int64_t)d * nb + blockIdx.x];
    for (int w = 0; w < 4; ++w) {
      const uint32_t c = cnt[w][d];
      cnt[w][d] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int it = 0; it < kIters; ++it) {
    const int64_t i = base + wave * kWaveKeys + it * 64 + lane;
    const bool ok = i < n;
    const uint32_t d = digit_of(kk[it], shift);
    const uint64_t valid = __builtin_amdgcn_ballot_w64(ok);
    const uint64_t peers = match_digit(d, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    uint32_t pos = 0;
    if (ok) pos = cnt[wave][d] + rank;
    __builtin_amdgcn_wave_barrier();
    if (ok) {
      kout[pos] = kk[it];
      vout[pos] = vv[it];
      if (rank == 0u) cnt[wave][d] = pos + (uint32_t)__popcll(peers);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ void k_hist_count(const uint32_t* n_dev, int64_t n_max, uint32_t* out) {
  if (threadIdx.x == 0) {
    const int64_t n = count_of(n_dev, n_max);
    *out = (uint32_t)(256 * ((n + kTile - 1) / kTile));
  }
}

struct Temp {
  uint32_t* hist;
  uint32_t* scan_tmp;
  uint32_t* n_hist;
  uint32_t* total;
};

Temp carve(void* temp, int64_t n_max) {
  const int64_t nb = (n_max + kTile - 1) / kTile;
  const int64_t nh = 256 * (nb > 0 ? nb : 1);
  char* p = (char*)temp;
  Temp t;
  t.hist = (uint32_t*)p; p += ((nh * 4 + 255) / 256) * 256;
  t.scan_tmp = (uint32_t*)p; p += ((scan_temp_bytes(nh) + 255) / 256) * 256;
  t.n_hist = (uint32_t*)p; p += 256;
  t.total = (uint32_t*)p;
  return t;
}

template <typename K>
void sort_impl(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, const uint32_t* n_dev,
               int64_t n_max, int begin_bit, int end_bit, void* temp, hipStream_t s, bool* in_alt) {
  *in_alt = false;
  if (n_max <= 0 || end_bit <= begin_bit) return;
  const int64_t nb = (n_max + kTile - 1) / kTile;
  Temp t = carve(temp, n_max);
  const uint32_t* nh_dev = nullptr;
  if (n_dev) {
    hipLaunchKernelGGL(k_hist_count, dim3(1), dim3(64), 0, s, n_dev, n_max, t.n_hist);
    nh_dev = t.n_hist;
  }
  K* kin = keys; uint32_t* vin = vals; K* kout = keys_alt; uint32_t* vout = vals_alt;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    hipLaunchKernelGGL(k_hist<K>, dim3((unsigned)nb), dim3(kThreads), 0, s, (const K*)kin, n_dev, n_max,
                       shift, t.hist);
    launch_scan(SCAN_VALUE, t.hist, nullptr, t.hist, t.total, nh_dev, 256 * nb, t.scan_tmp, s);
    hipLaunchKernelGGL(k_scatter<K>, dim3((unsigned)nb), dim3(kThreads), 0, s, (const K*)kin,
                       (const uint32_t*)vin, kout, vout, n_dev, n_max, shift, (const uint32_t*)t.hist);
    K* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
    *in_alt = !*in_alt;
  }
}

}  // namespace

size_t radix_temp_bytes(int64_t n_max) {
  const int64_t nb = (n_max + kTile - 1) / kTile;
  const int64_t nh = 256 * (nb > 0 ? nb : 1);
  return ((nh * 4 + 255) / 256) * 256 + ((scan_temp_bytes(nh) + 255) / 256) * 256 + 512;
}

void radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                    const uint32_t* n_dev, int64_t n_max, int begin_bit, int end_bit, void* temp,
                    hipStream_t s, bool* in_alt) {
  sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n_dev, n_max, begin_bit, end_bit, temp, s, in_alt);
}

void radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                    const uint32_t* n_dev, int64_t n_max, int begin_bit, int end_bit, void* temp,
                    hipStream_t s, bool* in_alt) {
  sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n_dev, n_max, begin_bit, end_bit, temp, s, in_alt);
}

}  // namespace lgs

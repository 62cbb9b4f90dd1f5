// Stable LSD radix sort of (key, u32 value) pairs on the device: the sort of
// visible Gaussians by depth and of (tile, Gaussian) pairs by tile that put
// every tile's list in front-to-back (depth, index) order.
//
// Per 8-bit digit pass: (1) per-block digit histogram, (2) per digit, an
// exclusive scan of its row of block counts and the digit's total (one
// work-group per digit), (3) stable scatter, each block adding the exclusive
// scan of the 256 digit totals to its row offsets.  Inside a block the
// rank of a key among equal digits comes from wave64 match masks: eight
// ballots give each lane the set of lanes holding its digit, the popcount of
// that set below the lane is its rank, and one leader lane per digit updates
// the running count.  No atomics, so the order is deterministic and stable.
#include "lgs_internal.h"

namespace lgs {
namespace {

constexpr int kThreads = 256;           // 4 waves
constexpr int kIters = 4;               // 64-key rows per wave
constexpr int kWaveKeys = 64 * kIters;  // 256
constexpr int kTile = 4 * kWaveKeys;    // 1024 keys per block (more blocks in flight: a pass over 1 M keys fills the chip)

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

// exclusive scan over the 256 threads of a block, in thread order
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* sh, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t v = sh[w];
    if (w < wave) pre += v;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return pre + inc - x;
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
  // all of the wave's keys are requested before the first is ranked
  // (unconditional loads at indices clamped to the last key)
  K kr[kIters];
#pragma unroll
  for (int it = 0; it < kIters; ++it) {
    const int64_t i = base + wave * kWaveKeys + it * 64 + lane;
    kr[it] = keys[i < n ? i : n - 1];
  }
#pragma unroll
  for (int it = 0; it < kIters; ++it) {
    const int64_t i = base + wave * kWaveKeys + it * 64 + lane;
    const bool ok = i < n;
    const uint32_t d = ok ? digit_of(kr[it], shift) : 0u;
    const uint64_t valid = __builtin_amdgcn_ballot_w64(ok);
    const uint64_t peers = match_digit(d, valid);
    if (ok && (peers & lt) == 0ull) cnt[wave][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  const int d = threadIdx.x;
  hist[(int64_t)d * nb + blockIdx.x] = cnt[0][d] + cnt[1][d] + cnt[2][d] + cnt[3][d];
}

constexpr int kRowItems = 8;

// One work-group per digit d: the row hist[d][0 .. nb) becomes its exclusive
// scan in place (the number of keys with digit d in the blocks before each
// block) and dtot[d] the digit's total.
__global__ void __launch_bounds__(kThreads) k_row_scan(const uint32_t* n_dev, int64_t n_max,
                                                       uint32_t* __restrict__ hist, uint32_t* __restrict__ dtot) {
  __shared__ uint32_t sh[kThreads / 64];
  const int64_t n = count_of(n_dev, n_max);
  const int64_t nb = (n + kTile - 1) / kTile;
  uint32_t* row = hist + (int64_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += (int64_t)kThreads * kRowItems) {
    const int64_t i0 = b0 + (int64_t)threadIdx.x * kRowItems;
    // every item requested before any is added (clamped unconditional loads)
    uint32_t v[kRowItems];
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) v[k] = row[i0 + k < nb ? i0 + k : nb - 1];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      v[k] = i0 + k < nb ? v[k] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_excl_scan256(sum, sh, tot);
#pragma unroll
    for (int k = 0; k < kRowItems; ++k) {
      if (i0 + k < nb) row[i0 + k] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

template <typename K>
__global__ void __launch_bounds__(kThreads) k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                      K* __restrict__ kout, uint32_t* __restrict__ vout,
                                                      const uint32_t* n_dev, int64_t n_max, int shift,
                                                      const uint32_t* __restrict__ off,
                                                      const uint32_t* __restrict__ dtot) {
  __shared__ uint32_t cnt[4][256];
  __shared__ uint32_t sh[kThreads / 64];
  const int64_t n = count_of(n_dev, n_max);
  const int64_t nb = (n + kTile - 1) / kTile;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  if (base >= n) return;
  // thread d's digit total and this block's row offset of digit d, requested
  // now (they do not depend on the keys)
  const uint32_t tot_d = dtot[threadIdx.x], off_d = off[(int64_t)threadIdx.x * nb + blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int d = threadIdx.x; d < 4 * 256; d += kThreads) (&cnt[0][0])[d] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  K kk[kIters];
  uint32_t vv[kIters];
  // all of the wave's keys and values are requested before the first key is
  // ranked (unconditional loads at indices clamped to the last key)
#pragma unroll
  for (int it = 0; it < kIters; ++it) {
    const int64_t i = base + wave * kWaveKeys + it * 64 + lane;
    const int64_t ic = i < n ? i : n - 1;
    kk[it] = kin[ic];
    vv[it] = vin[ic];
  }
#pragma unroll
  for (int it = 0; it < kIters; ++it) {
    const int64_t i = base + wave * kWaveKeys + it * 64 + lane;
    const bool ok = i < n;
    const uint32_t d = digit_of(kk[it], shift);
    const uint64_t valid = __builtin_amdgcn_ballot_w64(ok);
    const uint64_t peers = match_digit(d, valid);
    if (ok && (peers & lt) == 0ull) cnt[wave][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t all;
    // first position of digit d: the keys of smaller digits, then those of
    // digit d in earlier blocks
    uint32_t run = block_excl_scan256(tot_d, sh, all) + off_d;
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

struct Temp {
  uint32_t* hist;   // digit-major block counts, 256 x nb
  uint32_t* dtot;   // 256 digit totals
};

Temp carve(void* temp, int64_t n_max) {
  const int64_t nb = (n_max + kTile - 1) / kTile;
  const int64_t nh = 256 * (nb > 0 ? nb : 1);
  char* p = (char*)temp;
  Temp t;
  t.hist = (uint32_t*)p; p += ((nh * 4 + 255) / 256) * 256;
  t.dtot = (uint32_t*)p;
  return t;
}

template <typename K>
void sort_impl(K* keys, uint32_t* vals, K* keys_alt, uint32_t* vals_alt, const uint32_t* n_dev,
               int64_t n_max, int begin_bit, int end_bit, void* temp, hipStream_t s, bool* in_alt) {
  *in_alt = false;
  if (n_max <= 0 || end_bit <= begin_bit) return;
  const int64_t nb = (n_max + kTile - 1) / kTile;
  Temp t = carve(temp, n_max);
  K* kin = keys; uint32_t* vin = vals; K* kout = keys_alt; uint32_t* vout = vals_alt;
  for (int shift = begin_bit; shift < end_bit; shift += 8) {
    hipLaunchKernelGGL(k_hist<K>, dim3((unsigned)nb), dim3(kThreads), 0, s, (const K*)kin, n_dev, n_max,
                       shift, t.hist);
    hipLaunchKernelGGL(k_row_scan, dim3(256), dim3(kThreads), 0, s, n_dev, n_max, t.hist, t.dtot);
    hipLaunchKernelGGL(k_scatter<K>, dim3((unsigned)nb), dim3(kThreads), 0, s, (const K*)kin,
                       (const uint32_t*)vin, kout, vout, n_dev, n_max, shift, (const uint32_t*)t.hist,
                       (const uint32_t*)t.dtot);
    K* tk = kin; kin = kout; kout = tk;
    uint32_t* tv = vin; vin = vout; vout = tv;
    *in_alt = !*in_alt;
  }
}

}  // namespace

size_t radix_temp_bytes(int64_t n_max) {
  const int64_t nb = (n_max + kTile - 1) / kTile;
  const int64_t nh = 256 * (nb > 0 ? nb : 1);
  return ((nh * 4 + 255) / 256) * 256 + 256 * sizeof(uint32_t);
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

// Tile binning (the step between projection and compositing): device-wide
// exclusive scans, compaction of the visible (view, Gaussian) ids, the
// load-balanced emission of (tile, Gaussian) pairs in depth order, and the
// per-tile [start, end) ranges of the tile-sorted pair list.
//
// Every kernel reads its element count from device memory, so the same
// launches serve the eager path (grid sized to the exact count) and the
// captured graph (grid sized to a capacity; blocks past the count exit).
#include "lgs_internal.h"

namespace lgs {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;   // 2048

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// exclusive scan of one value per thread over a 256-thread block
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* sh, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(x, lane);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  uint32_t wsum = 0, tot = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    uint32_t s = sh[w];
    if (w < wave) wsum += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return wsum + inc - x;
}

__device__ __forceinline__ int64_t count_of(const uint32_t* n_dev, int64_t n_max) {
  return n_dev ? (int64_t)*n_dev : n_max;
}

// A gather scan reads src[idx[i]] at random once: the reduce pass leaves
// each gathered value in out[i], where the down-sweep reads it in order
// (and then overwrites it with the item's prefix).
//
// In both passes a thread requests all of its items' words before it uses
// any (unconditional loads at indices clamped to the last item, validity
// applied afterwards): a load under a bounds test that is used at once
// costs one memory round trip per item.
template <int MODE>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t* __restrict__ src,
                                                              const uint32_t* __restrict__ idx,
                                                              const uint32_t* n_dev, int64_t n_max,
                                                              uint32_t* __restrict__ bsum,
                                                              uint32_t* __restrict__ stash) {
  __shared__ uint32_t sh[4];
  const int64_t n = count_of(n_dev, n_max);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n) return;
  auto item = [&](int k) { return base + (int64_t)k * kScanThreads + threadIdx.x; };
  auto clamp = [&](int64_t i) { return i < n ? i : n - 1; };
  uint32_t x[kScanItems];
  if constexpr (MODE == SCAN_GATHER) {
    uint32_t id[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) id[k] = idx[clamp(item(k))];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) x[k] = src[id[k]];
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) x[k] = src[clamp(item(k))];
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = item(k);
    uint32_t v = MODE == SCAN_FLAG_NONZERO ? (x[k] != 0u ? 1u : 0u) : x[k];
    v = i < n ? v : 0u;
    if constexpr (MODE == SCAN_GATHER) {
      if (i < n) stash[i] = v;
    }
    s += v;
  }
  uint32_t total;
  block_excl_scan(s, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// one work-group scans the block sums in place (exclusive) and writes total

template <int MODE>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const uint32_t* __restrict__ src,
                                                            const uint32_t* __restrict__ idx,
                                                            const uint32_t* n_dev, int64_t n_max,
                                                            const uint32_t* __restrict__ bsum,
                                                            uint32_t* __restrict__ out, uint32_t* __restrict__ total,
                                                            uint32_t* __restrict__ out_at_idx, Compact cp) {
  __shared__ uint32_t sh[4];
  const int64_t n = count_of(n_dev, n_max);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (n == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *total = 0u;
    return;
  }
  if (base >= n) return;
  // thread t owns the contiguous items [base + t*8, base + t*8 + 8); their
  // words (the value, and the source index or depth key the writes below
  // need) are requested before the block sums, so all are in flight at once
  auto item = [&](int k) { return base + (int64_t)threadIdx.x * kScanItems + k; };
  auto clamp = [&](int64_t i) { return i < n ? i : n - 1; };
  uint32_t raw[kScanItems], aux[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t ic = clamp(item(k));
    raw[k] = MODE == SCAN_GATHER ? out[ic] : src[ic];
  }
  if (out_at_idx) {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) aux[k] = idx[clamp(item(k))];
  } else if (cp.ent) {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) aux[k] = cp.key_src[clamp(item(k))];
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) aux[k] = 0u;
  }
  asm volatile("" ::: "memory");
  // offset of this block: the sum of the block sums before it (each block
  // adds them up itself, so no separate pass over the block sums is needed)
  uint32_t pre = 0;
  for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kScanThreads) pre += bsum[b];
  uint32_t boff;
  block_excl_scan(pre, sh, boff);
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t x = MODE == SCAN_FLAG_NONZERO ? (raw[k] != 0u ? 1u : 0u) : raw[k];
    v[k] = item(k) < n ? x : 0u;
    s += v[k];
  }
  uint32_t btot;
  uint32_t run = block_excl_scan(s, sh, btot) + boff;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = item(k);
    if (i < n) {
      out[i] = run;
      if (out_at_idx) out_at_idx[aux[k]] = run;   // gather scans: the value also at its source index
      if (cp.ent && v[k] != 0u) {                  // flag scans: compaction of the flagged items
        cp.ent[run] = (uint32_t)i;
        cp.ent_copy[run] = (uint32_t)i;
        cp.keys[run] = aux[k];
      }
    }
    run += v[k];
  }
  if (base + kScanTile >= n && threadIdx.x == 0) *total = boff + btot;   // the last block
}

// reduce kernel must sum the same items as the down-sweep: both cover the
// block's 2048 items, only the assignment to threads differs.

constexpr int kEmitThreads = 256;
constexpr int kEmitPerThread = 4;
constexpr int kEmitTile = kEmitThreads * kEmitPerThread;   // 1024 pairs per block

// The first index i with a[i] > x (n if none) of a non-decreasing array,
// found by one wave: each step the 64 lanes probe 64 evenly
// spaced positions of the remaining range [lo, hi) and a ballot keeps the
// part holding the first element > x (hi stays a candidate: a[hi] > x or
// hi == n): about log64(n) dependent loads, where a one-thread binary
// search takes log2(n).
__device__ __forceinline__ int64_t wave_upper_bound_u32(const uint32_t* a, int64_t n, uint32_t x) {
  const int lane = threadIdx.x & 63;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t i = lo + (int64_t)lane * step;
    const bool valid = i < hi;
    const bool gt = valid && a[i] > x;
    const uint64_t m = __builtin_amdgcn_ballot_w64(gt);
    if (m != 0ull) {
      const int f = __builtin_ctzll(m);
      hi = lo + (int64_t)f * step;
      if (f > 0) lo += (int64_t)(f - 1) * step + 1;
    } else {
      const int last = 63 - __builtin_clzll(__builtin_amdgcn_ballot_w64(valid));
      lo += (int64_t)last * step + 1;
    }
  }
  return lo;
}

__global__ void __launch_bounds__(kEmitThreads) k_emit(
    const GeomRec* __restrict__ geom, const ViewDesc* __restrict__ views,
    const uint32_t* __restrict__ srid, const uint32_t* __restrict__ off_t,
    const Counters* __restrict__ cnt, int64_t cap_pairs, int npad_shift, int tile_shift,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
  __shared__ uint32_t s_off[kEmitTile + 2];
  __shared__ uint32_t s_rid[kEmitTile + 2];
  __shared__ int64_t s_j[2];
  const int64_t M = cnt->n_visible;
  const int64_t P = cnt->n_pairs;
  if (P > cap_pairs) return;                 // overflow: nothing valid is written
  const int64_t p0 = (int64_t)blockIdx.x * kEmitTile;
  if (p0 >= P) return;
  const int64_t p1 = (p0 + kEmitTile < P ? p0 + kEmitTile : P) - 1;   // last pair of the block
  // the entries owning the block's first and last pair: wave 0 and wave 1
  if (threadIdx.x < 128) {
    const int w = threadIdx.x >> 6;
    const int64_t j = wave_upper_bound_u32(off_t, M, (uint32_t)(w == 0 ? p0 : p1)) - 1;
    if ((threadIdx.x & 63) == 0) s_j[w] = j;
  }
  __syncthreads();
  const int64_t j0 = s_j[0], j1 = s_j[1];
  const int nj = (int)(j1 - j0 + 1);         // <= kEmitTile: every entry owns >= 1 pair
  for (int t = threadIdx.x; t < nj; t += kEmitThreads) {
    s_off[t] = off_t[j0 + t];
    s_rid[t] = srid[j0 + t];
  }
  __syncthreads();
  for (int k = 0; k < kEmitPerThread; ++k) {
    const int64_t pi = p0 + (int64_t)k * kEmitThreads + threadIdx.x;
    if (pi > p1) break;
    int lo = 0, hi = nj;                      // largest t with s_off[t] <= pi
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if ((int64_t)s_off[mid] <= pi) lo = mid; else hi = mid;
    }
    const uint32_t rid = s_rid[lo];
    const uint32_t local = (uint32_t)(pi - s_off[lo]);
    const uint32_t bb = geom[rid].bbox;
    const uint32_t tx0 = (bb & 255u) >> tile_shift, tx1 = ((bb >> 8) & 255u) >> tile_shift;
    const uint32_t ty0 = ((bb >> 16) & 255u) >> tile_shift;
    const uint32_t w = tx1 - tx0 + 1u;
    const uint32_t ty = ty0 + local / w, tx = tx0 + local % w;
    const ViewDesc& V = views[rid >> npad_shift];
    keys[pi] = (uint32_t)V.tile_off + ty * (uint32_t)V.tiles_x + tx;
    vals[pi] = rid;
  }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// two ranges of words zeroed by one launch
__global__ void __launch_bounds__(256) k_zero2_u32(uint32_t* __restrict__ p, int64_t np, uint32_t* __restrict__ q,
                                                   int64_t nq) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < np) p[i] = 0u;
  if (i < nq) q[i] = 0u;
}

__global__ void __launch_bounds__(256) k_fill_u8(uint8_t* __restrict__ p, uint8_t v,
                                                 const uint32_t* n_dev, int64_t n_max) {
  const int64_t n = count_of(n_dev, n_max);
  const int64_t i4 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (i4 + 3 < n) {
    const uint32_t w = (uint32_t)v * 0x01010101u;
    *(uint32_t*)(p + i4) = w;           // p is 4-byte aligned
  } else {
    for (int64_t i = i4; i < n; ++i) p[i] = v;
  }
}

__global__ void __launch_bounds__(256) k_tile_ranges(const uint32_t* __restrict__ keys,
                                                     const Counters* __restrict__ cnt,
                                                     uint2* __restrict__ ranges) {
  const int64_t P = cnt->overflow ? 0 : (int64_t)cnt->n_pairs;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= P) return;
  const uint32_t k = keys[i];
  if (i == 0 || keys[i - 1] != k) ranges[k].x = (uint32_t)i;
  if (i == P - 1 || keys[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
}

// The overflow flag and effective counts of the step, and (every thread) a
// range of words zeroed for the stages that follow.
__global__ void __launch_bounds__(256) k_set_overflow(Counters* cnt, uint64_t cap_pairs, uint64_t cap_slots,
                                                      uint32_t* __restrict__ zero, int64_t n_zero) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_zero; i += (int64_t)gridDim.x * 256) zero[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const bool ov = (uint64_t)cnt->n_pairs > cap_pairs || (uint64_t)cnt->n_slots > cap_slots;
    cnt->overflow = ov ? 1u : 0u;
    cnt->n_pairs_eff = ov ? 0u : cnt->n_pairs;
    cnt->n_slots_eff = ov ? 0u : cnt->n_slots;
  }
}

// Work items grouped by queue and, inside a queue, by descending list length
// (longest first): one work-group per queue, a counting sort of the queue's
// tiles on 256 length buckets (255 - bucket, bucket = 4 sqrt(length)
// clamped at 255) into the queue's segment of the output (a queue's items
// keep the segment the static table gives them).  Tiles of one bucket may
// come out in any order; the order only affects scheduling, not results.
constexpr int kOrderThreads = 256;
constexpr uint32_t kMaxTileItems = 16;   // 8x8 blocks of a 32-pixel tile

__device__ __forceinline__ uint32_t tile_bin(const uint2* __restrict__ ranges, const TileItems& T) {
  const uint2 r = ranges[T.tile];
  const uint32_t bucket = min(255u, (uint32_t)(4.f * sqrtf((float)(r.y - r.x))));
  return 255u - bucket;
}

// Work-group q: tiles tq[q] .. tq[q + 1] of the queue-major tile table, items
// to out[qoff[q] ..]; each tile's blocks are copied as a run, so they stay
// together in the output and are taken up by the queue's waves side by side.
__global__ void __launch_bounds__(kOrderThreads) k_order_items(const uint2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ items,
                                                             const uint32_t* __restrict__ qoff,
                                                             const TileItems* __restrict__ tiles,
                                                             const uint32_t* __restrict__ tq,
                                                             uint32_t* __restrict__ out) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[kOrderThreads / 64];
  const uint32_t q = blockIdx.x, t0 = tq[q], t1 = tq[q + 1], base = qoff[q];
  hist[threadIdx.x] = 0u;
  __syncthreads();
  for (uint32_t i = t0 + threadIdx.x; i < t1; i += kOrderThreads) {
    const TileItems T = tiles[i];
    atomicAdd(&hist[tile_bin(ranges, T)], T.count);
  }
  __syncthreads();
  // exclusive scan of the 256 bins, one per thread
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t a = hist[threadIdx.x];
  uint32_t inc = a;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
  hist[threadIdx.x] = base + pre + inc - a;
  __syncthreads();
  // a tile has at most kMaxTileItems blocks: all of its loads are issued
  // before the first store (one memory round trip per tile)
  for (uint32_t i = t0 + threadIdx.x; i < t1; i += kOrderThreads) {
    const TileItems T = tiles[i];
    const uint32_t pos = atomicAdd(&hist[tile_bin(ranges, T)], T.count);
    uint32_t v[kMaxTileItems];
#pragma unroll
    for (uint32_t k = 0; k < kMaxTileItems; ++k) v[k] = k < T.count ? items[T.first + k] : 0u;
#pragma unroll
    for (uint32_t k = 0; k < kMaxTileItems; ++k)
      if (k < T.count) out[pos + k] = v[k];
  }
}

}  // namespace

size_t scan_temp_bytes(int64_t n) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  return (size_t)(nb > 0 ? nb : 1) * sizeof(uint32_t);
}

template <int MODE>
static void launch_scan_t(const uint32_t* src, const uint32_t* idx, uint32_t* out, uint32_t* total,
                   const uint32_t* n_dev, int64_t n_max, void* temp, hipStream_t s, uint32_t* out_at_idx,
                   Compact cp) {
  const int64_t nb = (n_max + kScanTile - 1) / kScanTile;
  uint32_t* bsum = (uint32_t*)temp;
  if (nb > 0)
    hipLaunchKernelGGL(k_scan_reduce<MODE>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src, idx, n_dev, n_max,
                       bsum, out);
  hipLaunchKernelGGL(k_scan_down<MODE>, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kScanThreads), 0, s, src, idx,
                     n_dev, n_max, (const uint32_t*)bsum, out, total, out_at_idx, cp);
}

void launch_scan(int mode, const uint32_t* src, const uint32_t* idx, uint32_t* out, uint32_t* total,
                 const uint32_t* n_dev, int64_t n_max, void* temp, hipStream_t s, uint32_t* out_at_idx,
                 Compact cp) {
  if (mode == SCAN_FLAG_NONZERO)
    launch_scan_t<SCAN_FLAG_NONZERO>(src, idx, out, total, n_dev, n_max, temp, s, out_at_idx, cp);
  else if (mode == SCAN_VALUE)
    launch_scan_t<SCAN_VALUE>(src, idx, out, total, n_dev, n_max, temp, s, out_at_idx, cp);
  else
    launch_scan_t<SCAN_GATHER>(src, idx, out, total, n_dev, n_max, temp, s, out_at_idx, cp);
}

void launch_emit(const GeomRec* geom, const ViewDesc* views, const uint32_t* srid, const uint32_t* off_t,
                 const Counters* cnt, int64_t pair_grid_max, int64_t cap_pairs, int npad_shift,
                 int tile_shift, uint32_t* keys, uint32_t* vals, hipStream_t s) {
  const int64_t blocks = (pair_grid_max + kEmitTile - 1) / kEmitTile;
  if (blocks <= 0) return;
  hipLaunchKernelGGL(k_emit, dim3((unsigned)blocks), dim3(kEmitThreads), 0, s, geom, views, srid, off_t,
                     cnt, cap_pairs, npad_shift, tile_shift, keys, vals);
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}

void launch_zero2_u32(uint32_t* p, int64_t np, uint32_t* q, int64_t nq, hipStream_t s) {
  const int64_t n = std::max(np, nq);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero2_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, np, q, nq);
}

void launch_fill_u8(uint8_t* p, uint8_t v, const uint32_t* n_dev, int64_t n_max, hipStream_t s) {
  if (n_max <= 0) return;
  const int64_t blocks = (n_max + 1023) / 1024;
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n_dev, n_max);
}

void launch_tile_ranges(const uint32_t* keys, const Counters* cnt, int64_t grid_max, uint2* ranges,
                        hipStream_t s) {
  if (grid_max <= 0) return;
  hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((grid_max + 255) / 256)), dim3(256), 0, s, keys,
                     cnt, ranges);
}

void launch_set_overflow(Counters* cnt, uint64_t cap_pairs, uint64_t cap_slots, uint32_t* zero, int64_t n_zero,
                         hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n_zero + 255) / 256, 1), 1024);
  hipLaunchKernelGGL(k_set_overflow, dim3((unsigned)blocks), dim3(256), 0, s, cnt, cap_pairs, cap_slots, zero,
                     n_zero);
}

uint32_t* launch_order_items(const uint2* ranges, const uint32_t* items, const uint32_t* qoff, const TileItems* tiles,
                             const uint32_t* tq, int64_t n_tiles, uint32_t* out, hipStream_t s) {
  if (n_tiles <= 0) return out;
  hipLaunchKernelGGL(k_order_items, dim3(kQueues), dim3(kOrderThreads), 0, s, ranges, items, qoff, tiles, tq, out);
  return out;
}

}  // namespace lgs

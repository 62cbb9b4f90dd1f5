// Language-guided pruning (Sec. III-C, Eq. (4)) and the geometric criteria
// it is combined with.  For each Gaussian i, its K nearest other Gaussians
// (Euclidean distance of the means, ties by index) are examined; a
// neighbour j is redundant when |p_i - p_j| < tau_dist, the cosine
// similarity of their language features exceeds tau_sim, and i dominates j
// (larger opacity logit, or equal logits and i < j), so that one Gaussian of
// a redundant pair survives.  Geometric: opacity below min_opacity, largest
// scale above max_scale, or a non-finite mean / logit / log-scale.
//
// Only neighbours closer than tau_dist can be redundant, so the K nearest
// that matter are the K nearest among those within tau_dist.  The means are
// bucketed in a uniform grid of cell side tau_dist (a 63-bit key of the cell
// coordinates, 21 bits per axis), sorted by key (LSD radix sort), and each
// Gaussian scans the 27 cells around its own: a binary search for each
// cell's run in the sorted keys, then every candidate's squared distance in
// FP64 (no contraction: (dx^2 + dy^2) + dz^2) against tau_dist^2, kept in a
// register-resident sorted list of the K best (distance, index) pairs.  The
// similarity of each kept neighbour is evaluated in FP64 and the dominated
// neighbour's byte is set to 1 (every writer stores the same value).
#include "lgs_internal.h"

namespace lgs {
namespace {

constexpr int kPruneKMax = 32;
constexpr uint64_t kNoCell = ~0ull;
constexpr int64_t kCellBias = 1ll << 20;   // cell coordinates in [-2^20, 2^20)

__device__ __forceinline__ bool finite3(float x, float y, float z) {
  return isfinite(x) && isfinite(y) && isfinite(z);
}

__device__ __forceinline__ uint64_t cell_key(int64_t cx, int64_t cy, int64_t cz) {
  return ((uint64_t)(cx + kCellBias) << 42) | ((uint64_t)(cy + kCellBias) << 21) | (uint64_t)(cz + kCellBias);
}

__device__ __forceinline__ bool cell_ok(int64_t c) { return c >= -kCellBias && c < kCellBias; }

// Cell keys, indices and the geometric flags; a finite mean outside the
// grid's range sets *range_err.
__global__ void k_prune_keys(PruneArgs a, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                             uint8_t* __restrict__ geo, uint32_t* __restrict__ range_err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float x = a.means[i], y = a.means[a.n + i], z = a.means[2 * a.n + i];
  const float lam = a.logits[i];
  const float s0 = a.log_scales[i], s1 = a.log_scales[a.n + i], s2 = a.log_scales[2 * a.n + i];
  const bool fin = finite3(x, y, z) && isfinite(lam) && finite3(s0, s1, s2);
  const double smax = fmax(fmax((double)s0, (double)s1), (double)s2);
  geo[i] = (!fin || (double)lam < a.logit_min || smax > a.log_scale_max) ? 1 : 0;
  uint64_t key = kNoCell;
  if (finite3(x, y, z)) {
    const int64_t cx = (int64_t)floor((double)x * a.inv_cell), cy = (int64_t)floor((double)y * a.inv_cell),
                  cz = (int64_t)floor((double)z * a.inv_cell);
    if (cell_ok(cx) && cell_ok(cy) && cell_ok(cz)) key = cell_key(cx, cy, cz);
    else *range_err = 1u;
  }
  keys[i] = key;
  vals[i] = (uint32_t)i;
}

__device__ __forceinline__ float feat_at(const void* f, int bf16, int64_t n, int k, uint32_t g) {
  if (bf16) return __uint_as_float((uint32_t)((const unsigned short*)f)[(size_t)k * n + g] << 16);
  return ((const float*)f)[(size_t)k * n + g];
}

// first index in [lo, hi) whose key is >= key (keys sorted ascending)
__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* __restrict__ keys, int64_t lo, int64_t hi,
                                                   uint64_t key) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void k_prune_knn(PruneArgs a, const uint64_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ vals, uint8_t* __restrict__ sem) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n) return;
  const uint64_t key = keys[s];
  if (key == kNoCell) return;
  const uint32_t i = vals[s];
  const int64_t n = a.n;
  const double px = a.means[i], py = a.means[n + i], pz = a.means[2 * n + i];
  const int64_t cx = (int64_t)(key >> 42) - kCellBias, cy = (int64_t)((key >> 21) & 0x1fffffu) - kCellBias,
                cz = (int64_t)(key & 0x1fffffu) - kCellBias;
  // the K best (squared distance, index) pairs, ascending; unused = +inf
  double bd[kPruneKMax];
  uint32_t bj[kPruneKMax];
#pragma unroll
  for (int m = 0; m < kPruneKMax; ++m) {
    bd[m] = INFINITY;
    bj[m] = 0xffffffffu;
  }
  const double tau2 = a.tau2;
  // the three cells (ux, uy, cz - 1 .. cz + 1) have consecutive keys, so
  // their Gaussians form one run of the sorted array: 9 searches, not 27
  const int64_t uz0 = cz > -kCellBias ? cz - 1 : cz, uz1 = cz + 1 < kCellBias ? cz + 1 : cz;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
        const int64_t ux = cx + dx, uy = cy + dy;
        if (!cell_ok(ux) || !cell_ok(uy)) continue;
        const uint64_t k0 = cell_key(ux, uy, uz0), k1 = cell_key(ux, uy, uz1);
        for (int64_t t = lower_bound_u64(keys, 0, a.n_valid, k0); t < a.n_valid && keys[t] <= k1; ++t) {
          const uint32_t j = vals[t];
          if (j == i) continue;
          const double ex = (double)a.means[j] - px, ey = (double)a.means[n + j] - py,
                       ez = (double)a.means[2 * n + j] - pz;
          const double d2 = (ex * ex + ey * ey) + ez * ez;
          if (!(d2 < tau2)) continue;
          // insert into the sorted list: carry the candidate down, swapping
          // it with every entry it precedes (static indices: registers)
          double cd = d2;
          uint32_t cj = j;
#pragma unroll
          for (int m = 0; m < kPruneKMax; ++m) {
            const bool before = cd < bd[m] || (cd == bd[m] && cj < bj[m]);
            const double td = bd[m];
            const uint32_t tj = bj[m];
            bd[m] = before ? cd : td;
            bj[m] = before ? cj : tj;
            cd = before ? td : cd;
            cj = before ? tj : cj;
          }
        }
      }
  // similarity with each of the K nearest; mark the dominated neighbour
  double fi[16];
  double ni = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    fi[k] = feat_at(a.feat, a.feat_bf16, n, k, i);
    ni += fi[k] * fi[k];
  }
  const float li = a.logits[i];
#pragma unroll 1
  for (int m = 0; m < a.k; ++m) {
    const uint32_t j = bj[m];
    if (j == 0xffffffffu) break;
    double dot = 0.0, nj = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const double fj = feat_at(a.feat, a.feat_bf16, n, k, j);
      dot += fi[k] * fj;
      nj += fj * fj;
    }
    const double den = sqrt(ni) * sqrt(nj);
    const double sim = den > 0.0 ? dot / den : 0.0;
    const float lj = a.logits[j];
    const bool dom = li > lj || (li == lj && i < j);
    if (sim > a.tau_sim && dom) sem[j] = 1;
  }
}
#pragma clang fp contract(on)

// mask = semantic | geometric << 1, and the three counts (integer sums:
// the result does not depend on the order of the atomics)
__global__ __launch_bounds__(256) void k_prune_final(int64_t n, const uint8_t* __restrict__ sem,
                                                     const uint8_t* __restrict__ geo, uint8_t* __restrict__ mask,
                                                     unsigned long long* __restrict__ counts) {
  __shared__ unsigned int c[3];
  if (threadIdx.x < 3) c[threadIdx.x] = 0u;
  __syncthreads();
  unsigned int a0 = 0, a1 = 0, a2 = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t sv = sem[i], gv = geo[i];
    mask[i] = (uint8_t)(sv | (gv << 1));
    a0 += sv;
    a1 += gv;
    a2 += (sv | gv) ? 1u : 0u;
  }
  atomicAdd(&c[0], a0);
  atomicAdd(&c[1], a1);
  atomicAdd(&c[2], a2);
  __syncthreads();
  if (threadIdx.x < 3) atomicAdd(&counts[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

__global__ void k_prune_count_valid(const uint64_t* __restrict__ keys, int64_t n, int64_t* __restrict__ n_valid) {
  // sorted keys: the invalid (all-ones) keys are last; binary search in one thread
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (keys[mid] < kNoCell) lo = mid + 1;
      else hi = mid;
    }
    *n_valid = lo;
  }
}

}  // namespace

int prune_k_max() { return kPruneKMax; }

size_t prune_temp_bytes(int64_t n) {
  const size_t r = radix_temp_bytes(n);
  return ((r + 255) / 256) * 256;
}

// Host side of one pruning pass: keys, sort, neighbour search, mask.  The
// number of Gaussians with a usable cell is read back once (the neighbour
// kernel's search range), as is the range flag.
void launch_prune_keys(const PruneArgs& a, uint64_t* keys, uint32_t* vals, uint8_t* geo, uint32_t* range_err,
                       hipStream_t s) {
  if (a.n > 0)
    hipLaunchKernelGGL(k_prune_keys, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, keys, vals, geo,
                       range_err);
}

void launch_prune_count_valid(const uint64_t* keys, int64_t n, int64_t* n_valid, hipStream_t s) {
  hipLaunchKernelGGL(k_prune_count_valid, dim3(1), dim3(64), 0, s, keys, n, n_valid);
}

void launch_prune_knn(const PruneArgs& a, const uint64_t* keys, const uint32_t* vals, uint8_t* sem, hipStream_t s) {
  if (a.n > 0 && a.n_valid > 0)
    hipLaunchKernelGGL(k_prune_knn, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, keys, vals, sem);
}

void launch_prune_final(int64_t n, const uint8_t* sem, const uint8_t* geo, uint8_t* mask,
                        unsigned long long* counts, hipStream_t s) {
  int64_t g = (n + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_prune_final, dim3((unsigned)g), dim3(256), 0, s, n, sem, geo, mask, counts);
}

}  // namespace lgs

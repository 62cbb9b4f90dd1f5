// Mapping loss of Eq. (1) with the D-SSIM term of the photometric loss, and
// its gradient with respect to the rendered images, in one pass per view:
//
//   L = w_rgb ((1 - lam) mean|I - I*| + lam (1 - SSIM(I, I*)))
//     + w_depth mean|D - D*| + w_feat mean|F - F*|
//
// SSIM uses an 11 x 11 Gaussian window (separable, 1-D weights passed in),
// zero padding at the image border and the constants C1, C2.  With the local
// statistics m_x = E[X], s_xx = E[X^2], s_xy = E[XY] (E = window-weighted
// mean), the SSIM map S(p) depends on X only through m_x, s_xx and s_xy at p,
// so the gradient of sum_p S(p) with respect to X(q) is
//
//   (G * dS/dm_x)(q) + 2 X(q) (G * dS/ds_xx)(q) + Y(q) (G * dS/ds_xy)(q)
//
// (G the same window; it is symmetric, so correlation and convolution agree
// and the zero-padded window is its own adjoint).  One work-group computes a
// 32 x 32 output tile of one colour channel: it stages X and Y over the tile
// plus two window radii in LDS, forms the five window sums with a horizontal
// then a vertical pass (each thread slides along a row or a column, keeping
// its inputs in registers), evaluates S and the three coefficient maps over
// the tile plus one radius, filters those the same way, and writes the
// gradient of the channel.  The depth and feature L1 terms are a separate
// streaming kernel (16-byte accesses, several loads in flight per thread, no
// LDS), so that neither kernel's resources limit the other's occupancy.
// Per-work-group sums of |I - I*|, S, |D - D*| and |F - F*| go to partial
// arrays; a third kernel adds them per view in a fixed order (FP64), so the
// loss values are deterministic.
#include "lgs_internal.h"

namespace lgs {
namespace {

constexpr int kLT = 32;             // output tile side
constexpr int kLR = kSsimRadius;    // window radius (11 taps)
constexpr int kLTaps = 2 * kLR + 1;
constexpr int kLA = kLT + 4 * kLR;  // 52: side of the staged input region
constexpr int kLB = kLT + 2 * kLR;  // 42: side of the statistics region
constexpr int kPA = kLA + 1;        // odd row pitches: column walks across
constexpr int kPB = kLB + 1;        // lanes hit distinct LDS banks
constexpr int kPC = kLT + 1;
constexpr int kLossThreads = 256;
// One LDS region, reused stage by stage (a barrier between a stage's last
// read of one array and the first write of the next): X, Y (2 x 52 x 53);
// the five horizontal sums (5 x 52 x 43); the coefficient maps (3 x 42 x 43)
// followed by their horizontal sums (3 x 42 x 33).  44.7 KB: three
// work-groups per CU.
constexpr int kMax2(int a, int b) { return a > b ? a : b; }
constexpr int kLdsFloats = kMax2(kMax2(2 * kLA * kPA, 5 * kLA * kPB), 3 * kLB * kPB + 3 * kLB * kPC);

static_assert(kLT * kLT == 1024, "tile pixel index uses 10 bits");
static_assert(kLossDfPixels == 256 * 8, "depth/feature kernel: 8 pixels per thread");
static_assert(kLossThreads == 256, "stage thread maps assume 256 threads");

__device__ __forceinline__ float sgnf(float d) { return d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f); }

__device__ __forceinline__ void block_sum2(float& a, float& b, float* red) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();   // red may still be read from a previous use
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  a = (red[0] + red[2]) + (red[4] + red[6]);
  b = (red[1] + red[3]) + (red[5] + red[7]);
}

__global__ __launch_bounds__(kLossThreads) void k_loss_rgb(const LossView* __restrict__ views, LossConsts k,
                                                           float2* __restrict__ partials) {
  __shared__ float lds[kLdsFloats];
  __shared__ float red[8];
  const int b = blockIdx.x, t = threadIdx.x;
  int v = 0;
  while (v + 1 < k.n_views && views[v + 1].blk_off <= b) ++v;
  const LossView V = views[v];
  const int local = b - V.blk_off, tile = local / 3, role = local - 3 * tile;
  const int ty = tile / V.tiles_x, tx = tile - ty * V.tiles_x;
  const int x0 = tx * kLT, y0 = ty * kLT, W = V.W, H = V.H;
  const size_t plane = (size_t)W * H;
  float acc0 = 0.f, acc1 = 0.f;
  {
    const float* __restrict__ X = V.x + (size_t)role * plane;
    const float* __restrict__ Y = V.xt + (size_t)role * plane;
    float* __restrict__ G = V.gx + (size_t)role * plane;
    if (!k.ssim) {
      for (int e = t; e < kLT * kLT; e += kLossThreads) {
        const int gy = y0 + (e >> 5), gx = x0 + (e & 31);
        if (gy < H && gx < W) {
          const size_t o = (size_t)gy * W + gx;
          const float d = X[o] - Y[o];
          G[o] = V.s_l1 * sgnf(d);
          acc0 += fabsf(d);
        }
      }
    } else {
      // (A) X, Y over the tile plus 2 radii (zeros outside the image)
      float* sx = lds;
      float* sy = lds + kLA * kPA;
      for (int e = t; e < kLA * kLA; e += kLossThreads) {
        const int r = e / kLA, q = e - r * kLA;
        const int gy = y0 - 2 * kLR + r, gx = x0 - 2 * kLR + q;
        float a = 0.f, c = 0.f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
          const size_t o = (size_t)gy * W + gx;
          a = X[o];
          c = Y[o];
        }
        sx[r * kPA + q] = a;
        sy[r * kPA + q] = c;
      }
      __syncthreads();
      // (B) horizontal window sums of X, Y, X^2, Y^2, XY: 52 rows x 42
      // statistics columns; thread = (row, segment of 11 columns), walking
      // its 21 inputs once (the three products per input, then 5 FMAs per
      // tap); results stay in registers until every thread has read X, Y
      float hb[11][5];
      const int rb = t % kLA, segb = t / kLA;
      const int jb0 = min(segb * 11, kLB - 11);   // the last segment overlaps
      if (t < 4 * kLA) {
#pragma unroll
        for (int o = 0; o < 11; ++o)
#pragma unroll
          for (int q = 0; q < 5; ++q) hb[o][q] = 0.f;
#pragma unroll
        for (int m = 0; m < 21; ++m) {
          const float a = sx[rb * kPA + jb0 + m], c = sy[rb * kPA + jb0 + m];
          const float pv[5] = {a, c, a * a, c * c, a * c};
#pragma unroll
          for (int o = 0; o < 11; ++o) {
            const int tap = m - o;
            if (tap >= 0 && tap < kLTaps) {
#pragma unroll
              for (int q = 0; q < 5; ++q) hb[o][q] = fmaf(k.w[tap], pv[q], hb[o][q]);
            }
          }
        }
      }
      __syncthreads();   // X, Y are dead: the sums take their place
      float* h5 = lds;
      if (t < 4 * kLA) {
#pragma unroll
        for (int o = 0; o < 11; ++o)
#pragma unroll
          for (int q = 0; q < 5; ++q) h5[(q * kLA + rb) * kPB + jb0 + o] = hb[o][q];
      }
      __syncthreads();
      // (C) vertical sums -> local statistics over the 42 x 42 statistics
      // region; SSIM and its three coefficient maps (zero outside the image),
      // written over the sums once every thread has read them
      float st5[7][5];
      const int jc = t % kLB, segc = t / kLB;
      const int ic0 = segc * 7;
      if (t < 6 * kLB) {
#pragma unroll
        for (int o = 0; o < 7; ++o)
#pragma unroll
          for (int q = 0; q < 5; ++q) st5[o][q] = 0.f;
#pragma unroll
        for (int ii = 0; ii < 17; ++ii) {
          float val[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) val[q] = h5[(q * kLA + ic0 + ii) * kPB + jc];
#pragma unroll
          for (int o = 0; o < 7; ++o) {
            const int tap = ii - o;
            if (tap >= 0 && tap < kLTaps) {
#pragma unroll
              for (int q = 0; q < 5; ++q) st5[o][q] = fmaf(k.w[tap], val[q], st5[o][q]);
            }
          }
        }
      }
      __syncthreads();
      float* cf = lds;
      if (t < 6 * kLB) {
        const int gx = x0 - kLR + jc;
        const bool jin = jc >= kLR && jc < kLR + kLT;
#pragma unroll
        for (int o = 0; o < 7; ++o) {
          const int i = ic0 + o, gy = y0 - kLR + i;
          float ca = 0.f, cb = 0.f, cc = 0.f;
          if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const float mx = st5[o][0], my = st5[o][1];
            const float vx = st5[o][2] - mx * mx, vy = st5[o][3] - my * my, cxy = st5[o][4] - mx * my;
            const float A1 = 2.f * mx * my + k.c1, A2 = 2.f * cxy + k.c2;
            const float B1 = mx * mx + my * my + k.c1, B2 = vx + vy + k.c2;
            // B1 >= C1 and B2 >= C2 (up to rounding of the variances): normal
            // positive numbers, for which the hardware reciprocal is within 1 ulp
            const float rB1 = __builtin_amdgcn_rcpf(B1), rB2 = __builtin_amdgcn_rcpf(B2), iB = rB1 * rB2;
            const float S = A1 * A2 * iB;
            ca = 2.f * my * (A2 - A1) * iB + 2.f * mx * S * (rB2 - rB1);   // dS/dm_x
            cb = -S * rB2;                                                  // dS/ds_xx
            cc = 2.f * A1 * iB;                                             // dS/ds_xy
            if (jin && i >= kLR && i < kLR + kLT) acc1 += S;
          }
          cf[(0 * kLB + i) * kPB + jc] = ca;
          cf[(1 * kLB + i) * kPB + jc] = cb;
          cf[(2 * kLB + i) * kPB + jc] = cc;
        }
      }
      __syncthreads();
      // (D) horizontal sums of the coefficient maps: 42 rows x 32 columns;
      // thread = (row, segment of 6 columns; the last overlaps), into the
      // space after the coefficient maps
      float* h3 = lds + 3 * kLB * kPB;
      if (t < 6 * kLB) {
        const int i = t % kLB, seg = t / kLB;
        const int j0 = min(seg * 6, kLT - 6);
        float cv[3][16];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int m = 0; m < 16; ++m) cv[q][m] = cf[(q * kLB + i) * kPB + j0 + m];
#pragma unroll
        for (int o = 0; o < 6; ++o)
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            float sum = 0.f;
#pragma unroll
            for (int m = 0; m < kLTaps; ++m) sum = fmaf(k.w[m], cv[q][o + m], sum);
            h3[(q * kLB + i) * kPC + j0 + o] = sum;
          }
      }
      __syncthreads();
      // (E) vertical sums -> filtered coefficients at the tile's pixels;
      // thread = (column, segment of 4 rows)
      {
        const int jj = t & 31, seg = t >> 5;
        const int i0 = seg * 4;
        float acc[4][3];
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
          for (int q = 0; q < 3; ++q) acc[o][q] = 0.f;
#pragma unroll
        for (int m = 0; m < 14; ++m) {
          float val[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) val[q] = h3[(q * kLB + i0 + m) * kPC + jj];
#pragma unroll
          for (int o = 0; o < 4; ++o) {
            const int tap = m - o;
            if (tap >= 0 && tap < kLTaps) {
#pragma unroll
              for (int q = 0; q < 3; ++q) acc[o][q] = fmaf(k.w[tap], val[q], acc[o][q]);
            }
          }
        }
        const int gx = x0 + jj;
#pragma unroll
        for (int o = 0; o < 4; ++o) {
          const int gy = y0 + i0 + o;
          if (gy < H && gx < W) {
            const size_t off = (size_t)gy * W + gx;
            const float xo = X[off], yo = Y[off];
            const float d = xo - yo;
            acc0 += fabsf(d);
            G[off] = V.s_l1 * sgnf(d) - V.s_ssim * (acc[o][0] + 2.f * xo * acc[o][1] + yo * acc[o][2]);
          }
        }
      }
    }
  }
  block_sum2(acc0, acc1, red);
  if (t == 0) partials[b] = make_float2(acc0, acc1);
}

// Depth and feature L1 terms: work-group = a run of kLossDfPixels pixels of
// one view, all 1 + D channels (depth, then the D feature planes); each thread
// takes 8 pixels per channel (two 16-byte vectors when the view allows it)
// and loads four channels ahead before it computes and stores them.
constexpr int kDfGroup = 4;

__global__ __launch_bounds__(256) void k_loss_df(const LossView* __restrict__ views, int n_views,
                                                 float2* __restrict__ partials) {
  __shared__ float red[8];
  const int b = blockIdx.x, t = threadIdx.x;
  int v = 0;
  while (v + 1 < n_views && views[v + 1].df_off <= b) ++v;
  const LossView V = views[v];
  const int64_t n = (int64_t)V.W * V.H;
  const int64_t p0 = (int64_t)(b - V.df_off) * kLossDfPixels;
  const int nch = 1 + V.nf;
  float acc0 = 0.f, acc1 = 0.f;
  if (V.vec4) {
    const int64_t n4 = n >> 2;
    const int64_t i0 = (p0 >> 2) + t, i1 = i0 + 256;
    const bool in0 = i0 < n4, in1 = i1 < n4;
    for (int c0 = 0; c0 < nch; c0 += kDfGroup) {
      float4 y[kDfGroup][2], r[kDfGroup][2];
#pragma unroll
      for (int u = 0; u < kDfGroup; ++u) {
        const int ch = c0 + u;
        y[u][0] = y[u][1] = r[u][0] = r[u][1] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ch < nch) {
          const float4* Y4 = (const float4*)(ch == 0 ? V.d : V.f + (size_t)(ch - 1) * n);
          const float4* R4 = (const float4*)(ch == 0 ? V.dt : V.ft + (size_t)(ch - 1) * n);
          if (in0) { y[u][0] = Y4[i0]; r[u][0] = R4[i0]; }
          if (in1) { y[u][1] = Y4[i1]; r[u][1] = R4[i1]; }
        }
      }
#pragma unroll
      for (int u = 0; u < kDfGroup; ++u) {
        const int ch = c0 + u;
        if (ch < nch) {
          float4* G4 = (float4*)(ch == 0 ? V.gd : V.gf + (size_t)(ch - 1) * n);
          const float sc = ch == 0 ? V.s_d : V.s_f;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float4 d = make_float4(y[u][h].x - r[u][h].x, y[u][h].y - r[u][h].y, y[u][h].z - r[u][h].z,
                                         y[u][h].w - r[u][h].w);
            const float a = (fabsf(d.x) + fabsf(d.y)) + (fabsf(d.z) + fabsf(d.w));
            if (ch == 0) acc0 += a;
            else acc1 += a;
            if (h == 0 ? in0 : in1)
              G4[h == 0 ? i0 : i1] = make_float4(sc * sgnf(d.x), sc * sgnf(d.y), sc * sgnf(d.z), sc * sgnf(d.w));
          }
        }
      }
    }
  } else {
    for (int c0 = 0; c0 < nch; c0 += kDfGroup) {
      float y[kDfGroup][8], r[kDfGroup][8];
#pragma unroll
      for (int u = 0; u < kDfGroup; ++u) {
        const int ch = c0 + u;
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const int64_t p = p0 + t + 256 * h;
          y[u][h] = r[u][h] = 0.f;
          if (ch < nch && p < n) {
            y[u][h] = ch == 0 ? V.d[p] : V.f[(size_t)(ch - 1) * n + p];
            r[u][h] = ch == 0 ? V.dt[p] : V.ft[(size_t)(ch - 1) * n + p];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kDfGroup; ++u) {
        const int ch = c0 + u;
        if (ch < nch) {
          float* G = ch == 0 ? V.gd : V.gf + (size_t)(ch - 1) * n;
          const float sc = ch == 0 ? V.s_d : V.s_f;
#pragma unroll
          for (int h = 0; h < 8; ++h) {
            const int64_t p = p0 + t + 256 * h;
            const float d = y[u][h] - r[u][h];
            if (ch == 0) acc0 += fabsf(d);
            else acc1 += fabsf(d);
            if (p < n) G[p] = sc * sgnf(d);
          }
        }
      }
    }
  }
  block_sum2(acc0, acc1, red);
  if (t == 0) partials[b] = make_float2(acc0, acc1);
}

// Per view: the four loss terms from the work-groups' partial sums, added in
// a fixed order in FP64.
__global__ __launch_bounds__(256) void k_loss_terms(const LossView* __restrict__ views, int ssim,
                                                    const float2* __restrict__ part_rgb,
                                                    const float2* __restrict__ part_df, float* __restrict__ terms) {
  __shared__ double red[4][256];
  const int v = blockIdx.x, t = threadIdx.x;
  const LossView V = views[v];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = t; i < V.n_blk; i += 256) {
    const float2 p = part_rgb[V.blk_off + i];
    s[0] += (double)p.x;
    s[1] += (double)p.y;
  }
  for (int i = t; i < V.n_df; i += 256) {
    const float2 p = part_df[V.df_off + i];
    s[2] += (double)p.x;
    s[3] += (double)p.y;
  }
  for (int q = 0; q < 4; ++q) red[q][t] = s[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
      for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + h];
    __syncthreads();
  }
  if (t == 0) {
    const double n = (double)V.W * (double)V.H;
    terms[4 * v + 0] = (float)(red[0][0] / (3.0 * n));
    terms[4 * v + 1] = ssim ? (float)(1.0 - red[1][0] / (3.0 * n)) : 0.f;
    terms[4 * v + 2] = (float)(red[2][0] / n);
    terms[4 * v + 3] = (float)(red[3][0] / ((double)V.nf * n));
  }
}

}  // namespace

int64_t loss_blocks(int W, int H) {
  return 3ll * ((W + kLT - 1) / kLT) * ((H + kLT - 1) / kLT);
}

int64_t loss_df_blocks(int W, int H) {
  return ((int64_t)W * H + kLossDfPixels - 1) / kLossDfPixels;
}

int loss_tiles_x(int W) { return (W + kLT - 1) / kLT; }

void launch_loss_rgb(const LossView* views, const LossConsts& k, int64_t n_blocks, float2* partials,
                     hipStream_t s) {
  if (n_blocks > 0)
    hipLaunchKernelGGL(k_loss_rgb, dim3((unsigned)n_blocks), dim3(kLossThreads), 0, s, views, k, partials);
}

void launch_loss_df(const LossView* views, int n_views, int64_t n_blocks, float2* partials, hipStream_t s) {
  if (n_blocks > 0)
    hipLaunchKernelGGL(k_loss_df, dim3((unsigned)n_blocks), dim3(256), 0, s, views, n_views, partials);
}

void launch_loss_terms(const LossView* views, int n_views, int ssim, const float2* part_rgb,
                       const float2* part_df, float* terms, hipStream_t s) {
  if (n_views > 0)
    hipLaunchKernelGGL(k_loss_terms, dim3(n_views), dim3(256), 0, s, views, ssim, part_rgb, part_df, terms);
}

}  // namespace lgs

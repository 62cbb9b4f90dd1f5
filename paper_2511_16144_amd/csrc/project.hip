// Per-Gaussian stages: projection (forward) and its exact backward.
//
// Forward (Sec. III-B.1: the Gaussians Theta = {p, q, s, alpha, c, f} are
// rendered with the usual 3D Gaussian Splatting rasterizer): activation, view
// transform, EWA screen covariance and conic, the cut-off box in 8x8 pixel
// blocks and in binning tiles, the 32-bit depth key, and the packed
// appearance record.  Backward: the chain rule from the per-Gaussian
// screen-space gradient (mean', conic, opacity, rgb, depth, feature) to
// (p, log s, q, logit, c, f) and to the pose twist of Sec. III-B.2.
//
// Both run one thread per Gaussian and loop over the views, so a batched
// call reads each Gaussian once.  They are memory-bound (about 44 B read per
// Gaussian plus 60-80 B written per visible (view, Gaussian)), so the
// arithmetic is done in FP64: the per-pixel FP32 stages then start from
// correctly rounded means, conics and depths, which keeps their discrete
// decisions (cut-offs, order) reproducible.
#include "lgs_internal.h"
#include <math.h>

namespace lgs {
namespace {

struct Proj {
  double s[3], qh[4], qn, o;
  double R[9];   // R(qh), row-major
  double M[9];   // R diag(s)
};

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// O1 - O3: activation, rotation, M = R(qh) diag(s).
__device__ void activate(const double p[3], const double ls[3], const double q[4],
                         double logit, Proj& P) {
  for (int k = 0; k < 3; ++k) P.s[k] = exp(ls[k]);
  P.qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double inv = 1.0 / P.qn;
  for (int k = 0; k < 4; ++k) P.qh[k] = q[k] * inv;
  P.o = 1.0 / (1.0 + exp(-logit));
  const double w = P.qh[0], x = P.qh[1], y = P.qh[2], z = P.qh[3];
  P.R[0] = 1.0 - 2.0 * (y * y + z * z); P.R[1] = 2.0 * (x * y - w * z); P.R[2] = 2.0 * (x * z + w * y);
  P.R[3] = 2.0 * (x * y + w * z); P.R[4] = 1.0 - 2.0 * (x * x + z * z); P.R[5] = 2.0 * (y * z - w * x);
  P.R[6] = 2.0 * (x * z - w * y); P.R[7] = 2.0 * (y * z + w * x); P.R[8] = 1.0 - 2.0 * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P.M[3 * i + j] = P.R[3 * i + j] * P.s[j];
}

struct Screen {
  double xc[3];        // camera-space mean
  double mu[2];        // mean' (pixels)
  double J[6];         // 2x3 Jacobian (row-major)
  bool clx, cly;       // clamp active (x, y)
  double Lcx, Lcy;     // clamped x/z, y/z when active
  double Sc[9];        // camera-space covariance W Sigma W^T
  double a, b, c, det; // Sigma' = [[a, b], [b, c]]
};

// O4 - O8 for one view.
__device__ void to_screen(const ViewDesc& V, const double p[3], const Proj& P, double eps2d,
                          Screen& S) {
  for (int i = 0; i < 3; ++i)
    S.xc[i] = V.R[3 * i] * p[0] + V.R[3 * i + 1] * p[1] + V.R[3 * i + 2] * p[2] + V.t[i];
  const double z = S.xc[2];
  const double u = S.xc[0] / z, v = S.xc[1] / z;
  S.mu[0] = V.fx * u + V.cx;
  S.mu[1] = V.fy * v + V.cy;
  S.clx = fabs(u) > V.limx;
  S.cly = fabs(v) > V.limy;
  S.Lcx = fmin(fmax(u, -V.limx), V.limx);
  S.Lcy = fmin(fmax(v, -V.limy), V.limy);
  S.J[0] = V.fx / z; S.J[1] = 0.0; S.J[2] = -V.fx * S.Lcx / z;
  S.J[3] = 0.0; S.J[4] = V.fy / z; S.J[5] = -V.fy * S.Lcy / z;
  // WM = W M (3x3), m = J WM (2x3)
  double WM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      WM[3 * i + j] = V.R[3 * i] * P.M[j] + V.R[3 * i + 1] * P.M[3 + j] + V.R[3 * i + 2] * P.M[6 + j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S.Sc[3 * i + j] = WM[3 * i] * WM[3 * j] + WM[3 * i + 1] * WM[3 * j + 1] + WM[3 * i + 2] * WM[3 * j + 2];
  double m1[3], m2[3];
  for (int j = 0; j < 3; ++j) {
    m1[j] = S.J[0] * WM[j] + S.J[2] * WM[6 + j];
    m2[j] = S.J[4] * WM[3 + j] + S.J[5] * WM[6 + j];
  }
  S.a = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2] + eps2d;
  S.c = m2[0] * m2[0] + m2[1] * m2[1] + m2[2] * m2[2] + eps2d;
  S.b = m1[0] * m2[0] + m1[1] * m2[1] + m1[2] * m2[2];
  S.det = S.a * S.c - S.b * S.b;
}

// RGB and the first feature group (nfeat <= 16 channels; the rest 0)
template <bool BF16>
__device__ void load_app(const void* rgb, const void* feat, int64_t n, int64_t g, int nfeat, float y[20]) {
  if (BF16) {
    const uint16_t* r = (const uint16_t*)rgb;
    const uint16_t* f = (const uint16_t*)feat;
    for (int k = 0; k < 3; ++k) y[k] = __uint_as_float((uint32_t)r[k * n + g] << 16);
    for (int k = 0; k < 16; ++k) y[4 + k] = k < nfeat ? __uint_as_float((uint32_t)f[k * n + g] << 16) : 0.f;
  } else {
    const float* r = (const float*)rgb;
    const float* f = (const float*)feat;
    for (int k = 0; k < 3; ++k) y[k] = r[k * n + g];
    for (int k = 0; k < 16; ++k) y[4 + k] = k < nfeat ? f[k * n + g] : 0.f;
  }
  y[3] = 0.f;
}

// every feature plane of Gaussian g is finite (all D of them)
template <bool BF16>
__device__ bool feat_finite(const void* feat, int64_t n, int64_t g, int D) {
  bool fin = true;
  for (int k = 0; k < D; ++k) {
    const float x = BF16 ? __uint_as_float((uint32_t)((const uint16_t*)feat)[k * n + g] << 16)
                         : ((const float*)feat)[k * n + g];
    fin &= isfinite(x);
  }
  return fin;
}

// Sort key of a visible Gaussian's camera depth z > z_near: the FP64 bit
// pattern relative to z_near's, keeping 28 mantissa bits (depths closer than
// about 2^-28 relative share a key and keep index order; the sort is stable),
// clamped at z_near * 2^16.  Monotone in z, so sorting the keys sorts by depth.
__device__ __forceinline__ uint32_t depth_key(double z, double z_near) {
  const uint64_t d = (uint64_t)__double_as_longlong(z) - (uint64_t)__double_as_longlong(z_near);
  const uint64_t k = d >> 24;
  return k > 0xffffffffull ? 0xffffffffu : (uint32_t)k;
}

template <bool BF16>
__global__ void __launch_bounds__(256) k_project(
    Settings st, const ViewDesc* __restrict__ views, int n_views,
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const void* __restrict__ rgb, const void* __restrict__ feat, int64_t n, uint32_t npad_shift,
    GeomRec* __restrict__ geom, uint32_t* __restrict__ cnt_t, uint32_t* __restrict__ cnt_b,
    uint32_t* __restrict__ dkey, void* __restrict__ app, Counters* __restrict__ cnt) {
  // the step's counters start at zero (the first kernel of the step; no
  // kernel before it in the step reads them)
  if (blockIdx.x == 0)
    for (uint32_t i = threadIdx.x; i < sizeof(Counters) / 4; i += blockDim.x) ((uint32_t*)cnt)[i] = 0u;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ((int64_t)1 << npad_shift)) return;
  if (g >= n) {   // padding ids of the (view, Gaussian) index space: nothing visible
    for (int v = 0; v < n_views; ++v) {
      const uint64_t rid = ((uint64_t)v << npad_shift) | (uint64_t)g;
      cnt_t[rid] = 0;
      cnt_b[rid] = 0;
    }
    return;
  }
  double p[3], ls[3], q[4];
  for (int k = 0; k < 3; ++k) p[k] = means[k * n + g];
  for (int k = 0; k < 3; ++k) ls[k] = log_scales[k * n + g];
  for (int k = 0; k < 4; ++k) q[k] = quats[k * n + g];
  const double logit = logits[g];
  bool ok = finite_d(logit);
  for (int k = 0; k < 3; ++k) ok &= finite_d(p[k]) && finite_d(ls[k]);
  for (int k = 0; k < 4; ++k) ok &= finite_d(q[k]);
  ok &= (q[0] != 0.0 || q[1] != 0.0 || q[2] != 0.0 || q[3] != 0.0);
  Proj P;
  if (ok) activate(p, ls, q, logit, P);
  // the bbox is grown so that it holds every pixel an FP32 evaluation of the
  // cut-off tests could accept (relative 1e-5 on r^2, 1e-3 px absolute)
  const double lnmin = log((double)st.alpha_min);
  bool any_vis = false;
  for (int v = 0; v < n_views; ++v) {
    const ViewDesc V = views[v];
    const uint64_t rid = ((uint64_t)v << npad_shift) | (uint64_t)g;
    uint32_t ct = 0, cb = 0;
    if (ok) {
      Screen S;
      to_screen(V, p, P, (double)st.eps2d, S);
      const double z = S.xc[2];
      const double r2 = fmin((double)st.cutoff2, 2.0 * (log(P.o) - lnmin));
      bool vis = (z > (double)st.z_near) && (P.o >= (double)st.alpha_min) && isfinite(S.det) &&
                 isfinite(S.mu[0]) && isfinite(S.mu[1]) && S.det > 0.0;
      if (vis) {
        const double r2p = r2 * (1.0 + 1e-5) + 1e-4;
        const double rx = sqrt(r2p * S.a) + 1e-3, ry = sqrt(r2p * S.c) + 1e-3;
        const double fx0 = ceil(S.mu[0] - rx), fx1 = floor(S.mu[0] + rx);
        const double fy0 = ceil(S.mu[1] - ry), fy1 = floor(S.mu[1] + ry);
        vis = (fx0 <= (double)(V.W - 1)) && (fx1 >= 0.0) && (fy0 <= (double)(V.H - 1)) &&
              (fy1 >= 0.0) && fx0 <= fx1 && fy0 <= fy1;
        int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
        if (vis) {   // all four bounds now lie within the image after clamping
          x0 = (int)fmax(fx0, 0.0); x1 = (int)fmin(fx1, (double)(V.W - 1));
          y0 = (int)fmax(fy0, 0.0); y1 = (int)fmin(fy1, (double)(V.H - 1));
        }
        if (vis) {
          const int bx0 = x0 >> 3, bx1 = x1 >> 3, by0 = y0 >> 3, by1 = y1 >> 3;
          const int sh = st.tile_shift;
          ct = (uint32_t)(((bx1 >> sh) - (bx0 >> sh) + 1) * ((by1 >> sh) - (by0 >> sh) + 1));
          cb = (uint32_t)((bx1 - bx0 + 1) * (by1 - by0 + 1));
          GeomRec r;
          const double inv = 1.0 / S.det;
          r.mx = (float)(S.mu[0] - 8.0 * bx0);
          r.my = (float)(S.mu[1] - 8.0 * by0);
          r.qa = (float)(S.c * inv);
          r.qb2 = (float)(-2.0 * S.b * inv);
          r.qc = (float)(S.a * inv);
          r.o = (float)P.o;
          r.z = (float)z;
          r.bbox = (uint32_t)bx0 | ((uint32_t)bx1 << 8) | ((uint32_t)by0 << 16) | ((uint32_t)by1 << 24);
          geom[rid] = r;
          dkey[rid] = depth_key(z, (double)st.z_near);
          any_vis = true;
        }
      }
    }
    cnt_t[rid] = ct;
    cnt_b[rid] = cb;
  }
  if (!any_vis) return;
  float y[20];
  load_app<BF16>(rgb, feat, n, g, st.nfeat, y);
  bool fin = true;
  for (int k = 0; k < 4; ++k) fin &= isfinite(y[k]);
  fin &= feat_finite<BF16>(feat, n, g, st.feat_dim);
  if (!fin) {   // a non-finite colour or feature culls the Gaussian everywhere
    for (int v = 0; v < n_views; ++v) {
      const uint64_t rid = ((uint64_t)v << npad_shift) | (uint64_t)g;
      cnt_t[rid] = 0;
      cnt_b[rid] = 0;
    }
    return;
  }
  if (BF16) {
    const uint16_t* r = (const uint16_t*)rgb;
    const uint16_t* f = (const uint16_t*)feat;
    uint32_t w[10];
    w[0] = (uint32_t)r[g] | ((uint32_t)r[n + g] << 16);
    w[1] = (uint32_t)r[2 * n + g];
    for (int k = 0; k < 8; ++k) {
      const uint32_t lo = 2 * k < st.nfeat ? (uint32_t)f[(2 * k) * n + g] : 0u;
      const uint32_t hi = 2 * k + 1 < st.nfeat ? (uint32_t)f[(2 * k + 1) * n + g] : 0u;
      w[2 + k] = lo | (hi << 16);
    }
    uint32_t* dst = (uint32_t*)app + (size_t)g * 10;
    uint2* d2 = (uint2*)dst;
    for (int k = 0; k < 5; ++k) d2[k] = make_uint2(w[2 * k], w[2 * k + 1]);
  } else {
    float4* dst = (float4*)((float*)app + (size_t)g * 20);
    for (int k = 0; k < 5; ++k) dst[k] = make_float4(y[4 * k], y[4 * k + 1], y[4 * k + 2], y[4 * k + 3]);
  }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum_d(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// grad2d layout per visible (view, Gaussian): [Sx, Sy, Sxx, Sxy, Syy,
// opacity, r, g, b, z, f0..f15] (26 FP32), where S_* = sum over pixels of
// dL/dalpha * alpha times dx, dy, dx^2, dx dy, dy^2 (m2 = Q_xx dx^2 +
// 2 Q_xy dx dy + Q_yy dy^2, dx = pixel - mean, dL/dm2 = -1/2 dL/dalpha alpha):
// so dL/dQ_xx = -1/2 Sxx, dL/dQ_xy (the symmetric off-diagonal entry,
// counted twice in m2) = -Sxy, dL/dQ_yy = -1/2 Syy, and dL/dmean = Q (Sx, Sy).
// The per-view chain rule, one thread per visible (view, Gaussian) c (in
// (view, Gaussian) order, so a wave's 64 c belong to one view or a few
// consecutive ones): its contributions to dL/d(world mean), dL/dM and
// dL/dlogit go to contrib[c] (FP32, 16 floats: 3, 9, 1, pad), its pose-twist
// terms are summed per block of 64 c and view into twist_part[v][k][block].
// Every c of a view is visited by exactly one thread, with no divergence
// between views (one thread per Gaussian looping over the views ran the
// chain rule for every view a wave's Gaussians saw, with most lanes idle).
__global__ void __launch_bounds__(256) k_project_bwd_view(
    Settings st, const ViewDesc* __restrict__ views, const float* __restrict__ means,
    const float* __restrict__ log_scales, const float* __restrict__ quats, const float* __restrict__ logits,
    int64_t n, uint32_t npad_shift, const Counters* __restrict__ cnt, const uint32_t* __restrict__ ent,
    const float* __restrict__ grad2d, float* __restrict__ contrib, double* __restrict__ twist_part,
    int64_t nblk_max) {
  if (cnt->overflow) return;
  const int lane = threadIdx.x & 63;
  const uint32_t nv = cnt->n_visible;
  const int64_t nblk = ((int64_t)nv + 63) / 64;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int64_t w0 = __builtin_amdgcn_readfirstlane((int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const uint32_t gmask = (1u << npad_shift) - 1u;
  for (int64_t blk = w0; blk < nblk; blk += n_waves) {
    const int64_t ci = blk * 64 + lane;
    const bool act = ci < (int64_t)nv;
    uint32_t v = 0;
    double tw[6] = {0, 0, 0, 0, 0, 0};
    if (act) {
      const uint32_t rid = ent[ci];
      v = rid >> npad_shift;
      const int64_t g = rid & gmask;
      double p[3], ls[3], q[4];
      for (int k = 0; k < 3; ++k) p[k] = means[k * n + g];
      for (int k = 0; k < 3; ++k) ls[k] = log_scales[k * n + g];
      for (int k = 0; k < 4; ++k) q[k] = quats[k * n + g];
      Proj P;
      activate(p, ls, q, (double)logits[g], P);
      double gp[3] = {0, 0, 0}, gM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, glogit = 0.0;
      const ViewDesc V = views[v];
      const float* G = grad2d + (size_t)ci * kPartials;
      Screen S;
      to_screen(V, p, P, (double)st.eps2d, S);
      const double z = S.xc[2], iz = 1.0 / z;
      // conic -> Sigma':  G_Sigma' = -Q Gq Q  (symmetric representation)
      const double inv = 1.0 / S.det;
      const double Qa = S.c * inv, Qb = -S.b * inv, Qc = S.a * inv;
      const double ga_q = -0.5 * (double)G[2], gb_q = -0.5 * (double)G[3], gc_q = -0.5 * (double)G[4];
      // T1 = Gq Q
      const double t00 = ga_q * Qa + gb_q * Qb, t01 = ga_q * Qb + gb_q * Qc;
      const double t10 = gb_q * Qa + gc_q * Qb, t11 = gb_q * Qb + gc_q * Qc;
      const double s00 = -(Qa * t00 + Qb * t10), s01 = -(Qa * t01 + Qb * t11);
      const double s11 = -(Qb * t01 + Qc * t11);
      // Gsym = [[s00, s01], [s01, s11]]; Gc = J^T Gsym J (3x3)
      const double* J = S.J;
      double GJ[6];   // Gsym J (2x3)
      for (int j = 0; j < 3; ++j) {
        GJ[j] = s00 * J[j] + s01 * J[3 + j];
        GJ[3 + j] = s01 * J[j] + s11 * J[3 + j];
      }
      double Gc[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Gc[3 * i + j] = J[i] * GJ[j] + J[3 + i] * GJ[3 + j];
      // dL/dJ = 2 Gsym J Sc
      double dJ[6];
      for (int r = 0; r < 2; ++r)
        for (int j = 0; j < 3; ++j)
          dJ[3 * r + j] = 2.0 * (GJ[3 * r] * S.Sc[j] + GJ[3 * r + 1] * S.Sc[3 + j] + GJ[3 * r + 2] * S.Sc[6 + j]);
      // G_Sigma = W^T Gc W ; dL/dM += 2 G_Sigma M
      double GcW[9], GS[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          GcW[3 * i + j] = Gc[3 * i] * V.R[j] + Gc[3 * i + 1] * V.R[3 + j] + Gc[3 * i + 2] * V.R[6 + j];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          GS[3 * i + j] = V.R[i] * GcW[j] + V.R[3 + i] * GcW[3 + j] + V.R[6 + i] * GcW[6 + j];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          gM[3 * i + j] += 2.0 * (GS[3 * i] * P.M[j] + GS[3 * i + 1] * P.M[3 + j] + GS[3 * i + 2] * P.M[6 + j]);
      // camera-space mean gradient: mean', Jacobian, depth channel
      const double gmx = Qa * (double)G[0] + Qb * (double)G[1];
      const double gmy = Qb * (double)G[0] + Qc * (double)G[1];
      double gx[3];
      gx[0] = gmx * V.fx * iz;
      gx[1] = gmy * V.fy * iz;
      gx[2] = -(gmx * V.fx * S.xc[0] + gmy * V.fy * S.xc[1]) * iz * iz;
      gx[2] += -(dJ[0] * V.fx + dJ[4] * V.fy) * iz * iz;
      if (!S.clx) {   // J02 = -fx x / z^2
        gx[0] += dJ[2] * (-V.fx * iz * iz);
        gx[2] += dJ[2] * (2.0 * V.fx * S.xc[0] * iz * iz * iz);
      } else {        // J02 = -fx Lc / z
        gx[2] += dJ[2] * (V.fx * S.Lcx * iz * iz);
      }
      if (!S.cly) {
        gx[1] += dJ[5] * (-V.fy * iz * iz);
        gx[2] += dJ[5] * (2.0 * V.fy * S.xc[1] * iz * iz * iz);
      } else {
        gx[2] += dJ[5] * (V.fy * S.Lcy * iz * iz);
      }
      gx[2] += (double)G[9];
      for (int j = 0; j < 3; ++j) gp[j] += V.R[j] * gx[0] + V.R[3 + j] * gx[1] + V.R[6 + j] * gx[2];
      // twist: rho = gx; phi = xc x gx - 2 vee(Sc Gc - Gc Sc)
      tw[0] = gx[0]; tw[1] = gx[1]; tw[2] = gx[2];
      double A[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double s1 = 0, s2 = 0;
          for (int k = 0; k < 3; ++k) {
            s1 += S.Sc[3 * i + k] * Gc[3 * k + j];
            s2 += Gc[3 * i + k] * S.Sc[3 * k + j];
          }
          A[3 * i + j] = s1 - s2;
        }
      tw[3] = S.xc[1] * gx[2] - S.xc[2] * gx[1] - 2.0 * A[7];
      tw[4] = S.xc[2] * gx[0] - S.xc[0] * gx[2] - 2.0 * A[2];
      tw[5] = S.xc[0] * gx[1] - S.xc[1] * gx[0] - 2.0 * A[3];
      glogit += (double)G[5] * P.o * (1.0 - P.o);
      float* C = contrib + ci * 16;
      for (int k = 0; k < 3; ++k) C[k] = (float)gp[k];
      for (int k = 0; k < 9; ++k) C[3 + k] = (float)gM[k];
      C[12] = (float)glogit;
    }
    // the block's views: lane 0's (always a c of this block) to the last
    // active lane's; one partial per (view, component, block), in the order
    // of the blocks a view's c span
    const uint32_t vlo = __builtin_amdgcn_readfirstlane(v);
    uint32_t vmax = act ? v : 0u;
    for (int off = 32; off > 0; off >>= 1) vmax = max(vmax, (uint32_t)__shfl_xor((int)vmax, off, 64));
    const uint32_t vhi = __builtin_amdgcn_readfirstlane(vmax);
    for (uint32_t vv = vlo; vv <= vhi; ++vv) {
      const bool mine = act && v == vv;
      for (int k = 0; k < 6; ++k) {
        const double s = wave_sum_d(mine ? tw[k] : 0.0);
        if (lane == 0) twist_part[((int64_t)vv * 6 + k) * nblk_max + blk] = s;
      }
    }
  }
}

// Per Gaussian: the views' contributions summed in view order (a fixed
// order, so results are deterministic), then the activation's chain rule.
__global__ void __launch_bounds__(256) k_project_bwd(
    Settings st, int n_views, const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits, int64_t n,
    uint32_t npad_shift, const Counters* __restrict__ cnt, const uint32_t* __restrict__ cnt_t,
    const uint32_t* __restrict__ cidx, const float* __restrict__ grad2d, const float* __restrict__ contrib,
    float* __restrict__ g_means, float* __restrict__ g_ls, float* __restrict__ g_q, float* __restrict__ g_logit,
    float* __restrict__ g_rgb, float* __restrict__ g_feat) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = g < n;
  double p[3] = {0, 0, 0}, ls[3] = {0, 0, 0}, q[4] = {1, 0, 0, 0}, logit = 0.0;
  if (active) {
    for (int k = 0; k < 3; ++k) p[k] = means[k * n + g];
    for (int k = 0; k < 3; ++k) ls[k] = log_scales[k * n + g];
    for (int k = 0; k < 4; ++k) q[k] = quats[k * n + g];
    logit = logits[g];
  }
  Proj P;
  double gp[3] = {0, 0, 0}, gM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, glogit = 0.0;
  float gy[20];
  for (int k = 0; k < 20; ++k) gy[k] = 0.f;
  bool any = false;
  // views are taken 8 at a time with branch-free (clamped) loads, so that
  // their visibility and record index loads are in flight together
  constexpr int kVB = 8;
  if (active && cnt->overflow == 0u) {
    for (int v0 = 0; v0 < n_views; v0 += kVB) {
      uint32_t cix[kVB];
#pragma unroll
      for (int u = 0; u < kVB; ++u) {
        const uint64_t r = ((uint64_t)min(v0 + u, n_views - 1) << npad_shift) | (uint64_t)g;
        const uint32_t c = cnt_t[r], ci = cidx[r];
        cix[u] = (v0 + u < n_views && c != 0u) ? ci : ~0u;
      }
#pragma unroll
      for (int u = 0; u < kVB; ++u) {
        if (cix[u] == ~0u) continue;
        any = true;
        const float* C = contrib + (size_t)cix[u] * 16;
        for (int k = 0; k < 3; ++k) gp[k] += (double)C[k];
        for (int k = 0; k < 9; ++k) gM[k] += (double)C[3 + k];
        glogit += (double)C[12];
        const float* G = grad2d + (size_t)cix[u] * kPartials;
        for (int k = 0; k < 20; ++k) gy[k] += G[6 + k];
      }
    }
  }
  if (any) activate(p, ls, q, logit, P);
  if (!active) return;
  // M = R diag(s) -> s, R -> qh -> q
  double gls[3], gR[9];
  for (int j = 0; j < 3; ++j) {
    double gs = 0;
    for (int i = 0; i < 3; ++i) {
      gs += gM[3 * i + j] * (any ? P.R[3 * i + j] : 0.0);
      gR[3 * i + j] = gM[3 * i + j] * (any ? P.s[j] : 0.0);
    }
    gls[j] = any ? gs * P.s[j] : 0.0;
  }
  double gq[4] = {0, 0, 0, 0};
  if (any) {
    const double w = P.qh[0], x = P.qh[1], y = P.qh[2], zq = P.qh[3];
    double gw = 2.0 * (-zq * gR[1] + y * gR[2] + zq * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    double gxq = 2.0 * (y * gR[1] + zq * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] + zq * gR[6] +
                        w * gR[7] - 2.0 * x * gR[8]);
    double gyq = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + zq * gR[5] - w * gR[6] +
                        zq * gR[7] - 2.0 * y * gR[8]);
    double gzq = 2.0 * (-2.0 * zq * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * zq * gR[4] +
                        y * gR[5] + x * gR[6] + y * gR[7]);
    const double dot = w * gw + x * gxq + y * gyq + zq * gzq;
    const double iq = 1.0 / P.qn;
    gq[0] = (gw - w * dot) * iq;
    gq[1] = (gxq - x * dot) * iq;
    gq[2] = (gyq - y * dot) * iq;
    gq[3] = (gzq - zq * dot) * iq;
  }
  for (int k = 0; k < 3; ++k) g_means[k * n + g] = (float)gp[k];
  for (int k = 0; k < 3; ++k) g_ls[k * n + g] = (float)gls[k];
  for (int k = 0; k < 4; ++k) g_q[k * n + g] = (float)gq[k];
  g_logit[g] = (float)glogit;
  for (int k = 0; k < 3; ++k) g_rgb[k * n + g] = gy[k];
  for (int k = 0; k < 16; ++k)
    if (k < st.nfeat) g_feat[k * n + g] = gy[4 + k];
}

// Appearance records of a feature group beyond the first: RGB 0, slot 3
// unused, the group's nfeat feature planes starting at feat_g (the rest 0).
template <bool BF16>
__global__ void __launch_bounds__(256) k_pack_app_group(const void* __restrict__ feat_g, int nfeat, int64_t n,
                                                        void* __restrict__ app) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (BF16) {
    const uint16_t* f = (const uint16_t*)feat_g;
    uint32_t w[10];
    w[0] = 0u;
    w[1] = 0u;
    for (int k = 0; k < 8; ++k) {
      const uint32_t lo = 2 * k < nfeat ? (uint32_t)f[(2 * k) * n + g] : 0u;
      const uint32_t hi = 2 * k + 1 < nfeat ? (uint32_t)f[(2 * k + 1) * n + g] : 0u;
      w[2 + k] = lo | (hi << 16);
    }
    uint2* d2 = (uint2*)((uint32_t*)app + (size_t)g * 10);
    for (int k = 0; k < 5; ++k) d2[k] = make_uint2(w[2 * k], w[2 * k + 1]);
  } else {
    const float* f = (const float*)feat_g;
    float y[20];
    for (int k = 0; k < 4; ++k) y[k] = 0.f;
    for (int k = 0; k < 16; ++k) y[4 + k] = k < nfeat ? f[k * n + g] : 0.f;
    float4* dst = (float4*)((float*)app + (size_t)g * 20);
    for (int k = 0; k < 5; ++k) dst[k] = make_float4(y[4 * k], y[4 * k + 1], y[4 * k + 2], y[4 * k + 3]);
  }
}

// geo_acc[c][0..5] (=|+=) the geometric sums (moments, opacity) of
// a feature group's backward, per visible (view, Gaussian)
__global__ void __launch_bounds__(256) k_group_geo_acc(const float* __restrict__ grad2d_g,
                                                       const Counters* __restrict__ cnt,
                                                       float* __restrict__ geo_acc, int first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = (int64_t)cnt->n_visible * 6;
  if (i >= m || cnt->overflow) return;
  const int64_t c = i / 6, k = i - 6 * c;
  const float v = grad2d_g[(size_t)c * kPartials + k];
  geo_acc[i] = first ? v : geo_acc[i] + v;
}

__global__ void __launch_bounds__(256) k_group_geo_add(float* __restrict__ grad2d, const Counters* __restrict__ cnt,
                                                       const float* __restrict__ geo_acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = (int64_t)cnt->n_visible * 6;
  if (i >= m || cnt->overflow) return;
  const int64_t c = i / 6, k = i - 6 * c;
  grad2d[(size_t)c * kPartials + k] += geo_acc[i];
}

// a feature group's gradients: sum over the views where the Gaussian is
// visible of its colour partials f0.. (slots 10 ..), zero elsewhere
__global__ void __launch_bounds__(256) k_group_feat_grad(int n_views, int64_t n, uint32_t npad_shift,
                                                         const Counters* __restrict__ cnt,
                                                         const uint32_t* __restrict__ cnt_t,
                                                         const uint32_t* __restrict__ cidx,
                                                         const float* __restrict__ grad2d_g, int nfeat,
                                                         float* __restrict__ g_feat_g) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float acc[16];
  for (int k = 0; k < 16; ++k) acc[k] = 0.f;
  if (cnt->overflow == 0u)
    for (int v = 0; v < n_views; ++v) {
      const uint64_t rid = ((uint64_t)v << npad_shift) | (uint64_t)g;
      if (cnt_t[rid] != 0) {
        const float* G = grad2d_g + (size_t)cidx[rid] * kPartials;
        for (int k = 0; k < 16; ++k) acc[k] += G[10 + k];
      }
    }
  for (int k = 0; k < 16; ++k)
    if (k < nfeat) g_feat_g[k * n + g] = acc[k];
}

// twist[v][k] = sum over the projection-backward waves of their partial sums
// (stored [v][k][wave]); one workgroup per (view, component), fixed
// summation order.
// twist[v][k]: the block partials of view v's c range (the scan of the
// visibility flags gives its first c), summed in block order.
__global__ void __launch_bounds__(256) k_twist_final(const double* __restrict__ part, int64_t nblk_max,
                                                    int n_views, uint32_t npad_shift,
                                                    const uint32_t* __restrict__ cidx,
                                                    const Counters* __restrict__ cnt, float* __restrict__ twist) {
  __shared__ double red[256];
  const int idx = blockIdx.x;   // v * 6 + k
  const int v = idx / 6;
  double s = 0.0;
  if (cnt->overflow == 0u) {
    const int64_t c0 = cidx[(uint64_t)v << npad_shift];
    const int64_t c1 = v + 1 < n_views ? (int64_t)cidx[(uint64_t)(v + 1) << npad_shift] : (int64_t)cnt->n_visible;
    if (c1 > c0)
      for (int64_t b = c0 / 64 + threadIdx.x; b <= (c1 - 1) / 64; b += 256) s += part[(int64_t)idx * nblk_max + b];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) twist[idx] = (float)red[0];
}

}  // namespace

void launch_project(const Settings& st, const ViewDesc* views, int n_views, const float* means,
                    const float* log_scales, const float* quats, const float* logits,
                    const void* rgb, const void* feat, int app_bf16, int64_t n, uint32_t npad_shift,
                    GeomRec* geom, uint32_t* cnt_t, uint32_t* cnt_b, uint32_t* dkey, void* app,
                    Counters* cnt, hipStream_t s) {
  const int64_t npad = (int64_t)1 << npad_shift;
  const int blocks = (int)((npad + 255) / 256);
  if (app_bf16)
    hipLaunchKernelGGL(k_project<true>, dim3(blocks), dim3(256), 0, s, st, views, n_views, means,
                       log_scales, quats, logits, rgb, feat, n, npad_shift, geom, cnt_t, cnt_b, dkey, app, cnt);
  else
    hipLaunchKernelGGL(k_project<false>, dim3(blocks), dim3(256), 0, s, st, views, n_views, means,
                       log_scales, quats, logits, rgb, feat, n, npad_shift, geom, cnt_t, cnt_b, dkey, app, cnt);
}

void launch_pack_app_group(const void* feat_g, int nfeat, int app_bf16, int64_t n, void* app, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = (int)((n + 255) / 256);
  if (app_bf16) hipLaunchKernelGGL(k_pack_app_group<true>, dim3(blocks), dim3(256), 0, s, feat_g, nfeat, n, app);
  else hipLaunchKernelGGL(k_pack_app_group<false>, dim3(blocks), dim3(256), 0, s, feat_g, nfeat, n, app);
}

void launch_group_geo_acc(const float* grad2d_g, const Counters* cnt, int64_t n_max, float* geo_acc, int first,
                          hipStream_t s) {
  if (n_max <= 0) return;
  hipLaunchKernelGGL(k_group_geo_acc, dim3((unsigned)((6 * n_max + 255) / 256)), dim3(256), 0, s, grad2d_g, cnt,
                     geo_acc, first);
}

void launch_group_geo_add(float* grad2d, const Counters* cnt, int64_t n_max, const float* geo_acc, hipStream_t s) {
  if (n_max <= 0) return;
  hipLaunchKernelGGL(k_group_geo_add, dim3((unsigned)((6 * n_max + 255) / 256)), dim3(256), 0, s, grad2d, cnt,
                     geo_acc);
}

void launch_group_feat_grad(int n_views, int64_t n, uint32_t npad_shift, const Counters* cnt, const uint32_t* cnt_t,
                            const uint32_t* cidx, const float* grad2d_g, int nfeat, float* g_feat_g, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_group_feat_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_views, n, npad_shift,
                     cnt, cnt_t, cidx, grad2d_g, nfeat, g_feat_g);
}

// per-view contributions (16 floats per visible c) and the twist's block
// partials (n_views x 6 x blocks of 64 c), for at most n_rid visible c
size_t project_bwd_temp_bytes(int64_t n_rid, int n_views) {
  const int64_t nblk = (std::max<int64_t>(n_rid, 1) + 63) / 64;
  return (size_t)nblk * 64 * 16 * sizeof(float) + (size_t)nblk * n_views * 6 * sizeof(double);
}

void launch_project_bwd(const Settings& st, const ViewDesc* views, int n_views, const float* means,
                        const float* log_scales, const float* quats, const float* logits, int64_t n,
                        uint32_t npad_shift, int64_t n_rid, const Counters* cnt, const uint32_t* cnt_t,
                        const uint32_t* cidx, const uint32_t* ent, const float* grad2d, float* g_means,
                        float* g_ls, float* g_q, float* g_logit, float* g_rgb, float* g_feat, float* twist,
                        void* temp, hipStream_t s) {
  const int64_t nblk = (std::max<int64_t>(n_rid, 1) + 63) / 64;
  float* contrib = (float*)temp;
  double* tpart = (double*)((char*)temp + (size_t)nblk * 64 * 16 * sizeof(float));
  int dev = 0, cus = 256, occ = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_project_bwd_view, 256, 0);
  int64_t grid = (int64_t)cus * (occ > 0 ? occ : 1);
  const int64_t need = (nblk + 3) / 4;   // four waves (blocks of 64 c) per work-group
  if (grid > need) grid = need;
  hipLaunchKernelGGL(k_project_bwd_view, dim3((unsigned)grid), dim3(256), 0, s, st, views, means, log_scales,
                     quats, logits, n, npad_shift, cnt, ent, grad2d, contrib, tpart, nblk);
  const int blocks = (int)((n + 255) / 256);
  if (blocks > 0)
    hipLaunchKernelGGL(k_project_bwd, dim3(blocks), dim3(256), 0, s, st, n_views, means, log_scales, quats,
                       logits, n, npad_shift, cnt, cnt_t, cidx, grad2d, (const float*)contrib, g_means, g_ls,
                       g_q, g_logit, g_rgb, g_feat);
  if (twist)
    hipLaunchKernelGGL(k_twist_final, dim3(n_views * 6), dim3(256), 0, s, (const double*)tpart, nblk, n_views,
                       npad_shift, cidx, cnt, twist);
}

}  // namespace lgs

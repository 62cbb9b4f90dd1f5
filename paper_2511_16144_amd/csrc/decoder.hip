// Feature-distillation loss of Eq. (2) through a 1x1-convolution decoder, and
// its gradients, on the matrix cores:
//
//   Z(p) = W F(p) + b  (W [C][16], b [C], F [16][H][W]),
//   L = w_feat / (C H W) * sum_{c,p} |Z[c][p] - T[c][p]|   (T = F_gt, [C][H][W])
//   R = sign(Z - T);  dL/dF = s W^T R;  dL/dW = s R F^T;  dL/db = s sum_p R,
//   s = w_feat / (C H W).
//
// Three products per pixel with 16 or 32 as the inner dimension, so each is a
// run of v_mfma_f32_16x16x32_bf16 (FP32 accumulation).  The FP32 operands are
// split into two BF16 terms (x = x_hi + x_lo, 16 significant bits); R is
// -1, 0 or 1, exact in BF16.  Z^T = F^T W^T takes the two splits in one
// instruction pair: A = [F_hi | F_lo] (K = 32) against B = [W_hi ; W_hi], then
// A against [W_lo ; W_lo], i.e. all four products of the split operands.
//
// Work-group = 16 waves of 32 channels for C = 512 (four per SIMD, 128
// VGPRs each), 8 waves of 32 channels for C = 256; a work-group walks a
// contiguous run of 32-pixel chunks of one view (a fixed assignment, so its
// partial sums are deterministic), loading the next chunk's inputs while it
// works on one, with one work-group barrier per chunk.  Wave w owns the
// channels [32 w, 32 (w+1)): per chunk it
// forms its Z^T tiles (16 pixels x 16 channels; the pixel order of the rows
// gives lane l 8 consecutive pixels of one channel over the chunk's two
// column groups, so its targets are one 16-byte load per channel), the
// signs, its share of dL/dF (summed over the waves through LDS) and its
// rows of dL/dW and dL/db (kept in registers over all chunks).  A second
// kernel adds the work-groups' partials in a fixed order.
#include "lgs_internal.h"

#include <type_traits>

namespace lgs {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kChunk = 32;            // pixels per chunk
constexpr int kFA = 40;               // LDS pitch (u16) of the [pixel][k] F rows (80 B)
constexpr int kFT = 40;               // LDS pitch (u16) of the [feature][pixel] F rows
constexpr int kRC = 40;               // LDS pitch (u16) of the [channel][pixel] sign rows

__device__ __forceinline__ unsigned short to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8_t as_bf16x8(u16x8 v) { return __builtin_bit_cast(bf16x8_t, v); }

// Work-group barrier for LDS traffic: waits for this wave's LDS accesses
// only, so the prefetched global loads stay in flight across it (a full
// __syncthreads() also waits for every outstanding global load).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ f32x4 mfma(bf16x8_t a, bf16x8_t b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight consecutive targets as loaded (BF16: 16 bytes, FP32: 32 bytes),
// vector loads when aligned and in range, else element by element (zero past
// the end); unpacked to FP32 when used.
struct F8 { float4 a, b; };
template <typename T> struct Raw8;
template <> struct Raw8<unsigned short> { typedef uint4 type; };
template <> struct Raw8<float> { typedef F8 type; };

__device__ __forceinline__ uint4 load_raw8(const unsigned short* p, bool vec, int64_t left) {
  if (vec) return *(const uint4*)p;
  uint32_t h[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] = i < left ? (uint32_t)p[i] : 0u;
  return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}
__device__ __forceinline__ F8 load_raw8(const float* p, bool vec, int64_t left) {
  F8 r;
  if (vec) {
    r.a = *(const float4*)p;
    r.b = *(const float4*)(p + 4);
    return r;
  }
  float f[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) f[i] = i < left ? p[i] : 0.f;
  r.a = make_float4(f[0], f[1], f[2], f[3]);
  r.b = make_float4(f[4], f[5], f[6], f[7]);
  return r;
}
// targets h*4 .. h*4 + 3 of the eight
__device__ __forceinline__ void unpack4(uint4 v, int h, float t[4]) {
  const uint32_t x = h ? v.z : v.x, y = h ? v.w : v.y;
  t[0] = __uint_as_float(x << 16); t[1] = __uint_as_float(x & 0xffff0000u);
  t[2] = __uint_as_float(y << 16); t[3] = __uint_as_float(y & 0xffff0000u);
}
__device__ __forceinline__ void unpack4(const F8& v, int h, float t[4]) {
  const float4 u = h ? v.b : v.a;
  t[0] = u.x; t[1] = u.y; t[2] = u.z; t[3] = u.w;
}

// NT: 16-channel tiles per wave, NW: waves per work-group (C = 16 NT NW,
// NT >= 2); at most 1024 threads, so NW = 16 leaves 128 VGPRs per lane (four
// waves per SIMD) and NW = 8 leaves 256 (two)
template <typename TT, int NT, int NW>
__global__ __launch_bounds__(64 * NW) void k_decoder(DecArgs a, float* __restrict__ part) {
  constexpr int kDecWaves = NW;
  constexpr int kDecThreads = 64 * NW;
  constexpr int Cw = 16 * NT;             // channels per wave
  constexpr int KS = Cw / 32;             // 32-channel steps of the dF product
  static_assert(KS >= 1, "at least 32 channels per wave");
  // F rows and the waves' dF partials are double-buffered by chunk parity,
  // so that one work-group barrier per chunk suffices (see the loop)
  __shared__ __attribute__((aligned(16))) unsigned short fA[2][kChunk * kFA];     // [pixel][F_hi 16 | F_lo 16]
  __shared__ __attribute__((aligned(16))) unsigned short fT[2][2 * 16 * kFT];     // [hi/lo][feature][pixel]
  __shared__ __attribute__((aligned(16))) unsigned short rC[kDecWaves][Cw * kRC];      // [channel][pixel] signs
  // [pixel][channel] signs.  A wave's 2-byte sign stores hit four rows 8
  // apart at once (one per lane group), and with 16-byte-aligned rows those
  // always share banks, so each row's channels are rotated by Cw / 4
  // channels per group of 8 rows: the four lane groups then fall on disjoint
  // banks.  Readers take 8-channel runs, which the rotation keeps whole.
  constexpr int kRP = Cw + 8;
  auto rp_col = [&](int row, int col) { return (col + (Cw / 4) * ((row >> 3) & 3)) & (Cw - 1); };
  static_assert((Cw & (Cw - 1)) == 0 && Cw >= 32, "rotation modulo a power-of-two channel count");
  __shared__ __attribute__((aligned(16))) unsigned short rP[kDecWaves][kChunk * kRP];
  __shared__ __attribute__((aligned(16))) float dfr[2][kDecWaves * 16 * kChunk];      // [wave][feature][pixel]
  __shared__ float red[kDecWaves];

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int c0 = w * Cw;   // first channel of this wave
  // the view of this work-group (views own consecutive runs of work-groups)
  int vi = 0;
  for (int u = 1; u < a.n_views; ++u)
    if ((int)blockIdx.x >= a.v[u].g0) vi = u;
  const int64_t n = a.v[vi].n;
  const float* __restrict__ feat = a.v[vi].feat;
  const TT* __restrict__ target = (const TT*)a.v[vi].target;
  float* __restrict__ grad_feat = a.v[vi].grad_feat;
  const float scale = a.v[vi].scale;
  const bool vec = a.v[vi].vec != 0;

  // W is staged in LDS once (over the sign rows, unused until the first
  // chunk's first barrier), then every wave builds its operands from there
  // (C = 16 NT kDecWaves: every thread copies the same number of values,
  // all requested before the first is stored)
  float* wl = (float*)&rC[0][0];
  static_assert(sizeof(rC) >= (size_t)kDecWaves * Cw * 16 * sizeof(float), "W fits over the sign rows");
  {
    constexpr int kWv = kDecWaves * Cw * 16 / kDecThreads;   // values per thread
    static_assert(kWv * kDecThreads == kDecWaves * Cw * 16, "W divides evenly among the threads");
    float wv[kWv];
#pragma unroll
    for (int i = 0; i < kWv; ++i) wv[i] = a.weight[t + i * kDecThreads];
#pragma unroll
    for (int i = 0; i < kWv; ++i) wl[t + i * kDecThreads] = wv[i];
  }
  __syncthreads();
  // this wave's operands of W, split hi/lo, in registers for the whole run
  // Z^T B operand, tile nt: lane (k block q4, channel r16): [W_hi ; W_hi] and [W_lo ; W_lo]
  bf16x8_t bz1[NT], bz2[NT];
  float bias[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int ch = c0 + 16 * nt + r16;
    const float* wr = wl + ch * 16 + 8 * (q4 & 1);
    u16x8 h, l;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float x = wr[k];
      const unsigned short hi = to_bf16(x);
      h[k] = hi;
      l[k] = to_bf16(x - from_bf16(hi));
    }
    bz1[nt] = as_bf16x8(h);
    bz2[nt] = as_bf16x8(l);
    bias[nt] = a.bias[ch] + 0.f;   // +0 for a -0 bias: Z is then never -0
  }
  // dF A operand (W^T), step ks: lane (feature r16, channels 32 ks + 8 q4 .. + 7)
  bf16x8_t wt_h[KS], wt_l[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    u16x8 h, l;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int ch = c0 + 32 * ks + 8 * q4 + k;
      const float x = wl[ch * 16 + r16];
      const unsigned short hi = to_bf16(x);
      h[k] = hi;
      l[k] = to_bf16(x - from_bf16(hi));
    }
    wt_h[ks] = as_bf16x8(h);
    wt_l[ks] = as_bf16x8(l);
  }

  f32x4 dw[NT];            // dW^T tiles: lane (features 4 q4 + i, channel 16 nt + r16)
  int db[NT];              // per lane: channel 16 nt + r16, its pixels 4 q4 .. + 3 (sum of signs)
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    dw[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
    db[nt] = 0;
  }
  // BF16 targets: for Z^T row m of column group cg (pixel 8 (m / 4) + 4 cg
  // + m % 4) the A row that is -1 at that pixel's K index and 0 elsewhere;
  // lane (r16, q4) holds K indices 8 q4 .. 8 q4 + 7 of row r16
  constexpr bool kTsel = sizeof(TT) == 2;
  bf16x8_t tsel[2];
#pragma unroll
  for (int cg = 0; cg < 2; ++cg) {
    u16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = ((r16 >> 2) == q4 && j == 4 * cg + (r16 & 3)) ? (unsigned short)0xBF80u : 0;
    tsel[cg] = as_bf16x8(v);
  }
  float lsum = 0.f;

  // The targets and feature element of the next kDecPF chunks are loaded
  // into registers ahead of their use (kDecPF register sets, the chunk loop
  // unrolled by kDecPF so that each set stays in the same registers), so the
  // loads' latency overlaps the matrix products of the chunks before.  The
  // depth is what the register file holds without spilling: a chunk's
  // targets take 4 NT registers in BF16, 8 NT in FP32; at 16 waves (128
  // VGPRs) one chunk ahead.
  constexpr int kDecPF = NW == 16 ? 1 : (sizeof(TT) == 2 ? 3 : 2) - (NT == 4 ? 1 : 0);
  typedef typename Raw8<TT>::type RawT;
  RawT tr[kDecPF][NT];
  float fr[kDecPF];
  static_assert(kDecThreads >= 16 * kChunk, "at most one feature element per thread and chunk");
  const int fk = (t >> 5) & 15, fpx = t & 31;
  const bool fth = t < 16 * kChunk;   // the threads that carry the chunk's feature elements
  // lane (q4, r16) of the Z^T products holds pixels 8 q4 .. 8 q4 + 7 of the
  // chunk (rows 4 q4 .. 4 q4 + 3 of column group cg are pixels 8 q4 + 4 cg
  // + i): its targets of one channel are one 16-byte load
  auto fetch = [&](int64_t ck, RawT (&trs)[NT], float& frs) {
    const int64_t p0 = ck * kChunk;
    const bool full = p0 + kChunk <= n;
    frs = fth && p0 + fpx < n ? feat[(size_t)fk * n + p0 + fpx] : 0.f;
    const int64_t pp = p0 + 8 * q4;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const TT* tp = target + (size_t)(c0 + 16 * nt + r16) * n + pp;
      trs[nt] = load_raw8(tp, full && vec, n - pp);
    }
  };
  // each work-group takes a contiguous run of its view's chunks, so the two
  // halves of a 128-byte target line are read by the same work-group one
  // chunk apart
  const int64_t n_chunks = (n + kChunk - 1) / kChunk;
  const int64_t per = (n_chunks + a.v[vi].groups - 1) / a.v[vi].groups;
  const int64_t ck0 = (int64_t)((int)blockIdx.x - a.v[vi].g0) * per;
  const int64_t ck1 = ck0 + per < n_chunks ? ck0 + per : n_chunks;
  // chunk pc's dL/dF: the waves' partials (buffer par) summed in a fixed order
  auto store_df = [&](int64_t pc, int par) {
    const int64_t q0 = pc * kChunk;
    for (int e = t; e < 16 * kChunk; e += kDecThreads) {
      const int k = e >> 5, px = e & 31;
      float v = 0.f;
#pragma unroll
      for (int u = 0; u < kDecWaves; ++u) v += dfr[par][(u * 16 + k) * kChunk + px];
      if (q0 + px < n) grad_feat[(size_t)k * n + q0 + px] = scale * v;
    }
  };
  // one chunk; its inputs are in (cur, frc), which are refilled with chunk
  // ck + kDecPF's as soon as they have been used
  auto chunk = [&](int64_t ck, RawT (&cur)[NT], float& frc) {
    const int64_t p0 = ck * kChunk;
    const int par = (int)((ck - ck0) & 1);
    const unsigned short* fAc = fA[par];
    const unsigned short* fTc = fT[par];
    // (1) F chunk -> LDS: [pixel][F_hi | F_lo] and [hi/lo][feature][pixel]
    if (fth) {
      const unsigned short hi = to_bf16(frc), lo = to_bf16(frc - from_bf16(hi));
      fA[par][fpx * kFA + fk] = hi;
      fA[par][fpx * kFA + 16 + fk] = lo;
      fT[par][fk * kFT + fpx] = hi;
      fT[par][16 * kFT + fk * kFT + fpx] = lo;
    }
    // The one barrier of the chunk: the F rows of this chunk are complete, and
    // every wave has finished the previous chunk (its dF partials are in the
    // other buffer, and it no longer reads this buffer's F rows from two
    // chunks ago).  The sign rows are per wave and need no barrier.
    lds_barrier();
    if (ck > ck0) store_df(ck - 1, par ^ 1);
    // (2) Z^T tiles, signs, loss, db; signs to LDS in both layouts (a
    // chunk wholly inside the image skips the per-pixel validity tests)
    const int lim = n - p0 < kChunk ? (int)(n - p0) : kChunk;   // valid pixels of the chunk
    auto signs = [&](auto full_tag) {
      constexpr bool kFull = decltype(full_tag)::value;
#pragma unroll
    for (int cg = 0; cg < 2; ++cg) {
      // A row r16 of column group cg is pixel 8 (r16 / 4) + 4 cg + r16 % 4
      const bf16x8_t af = as_bf16x8(*(const u16x8*)(fAc + (8 * (r16 >> 2) + 4 * cg + (r16 & 3)) * kFA + 8 * q4));
      const int pl = 8 * q4 + 4 * cg;    // first of this lane's 4 pixels of this column group
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        f32x4 z = {bias[nt], bias[nt], bias[nt], bias[nt]};
        // BF16 targets enter the product as they are: the selector rows of
        // -1 pick each row's own target (one non-zero product, exact), so
        // the tile comes out as Z - T
        if constexpr (kTsel) z = mfma(tsel[cg], __builtin_bit_cast(bf16x8_t, cur[nt]), z);
        z = mfma(af, bz1[nt], z);
        z = mfma(af, bz2[nt], z);
        float tv[4];
        if constexpr (!kTsel) unpack4(cur[nt], cg, tv);
        uint32_t sb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool valid = kFull || pl + i < lim;
          const float d = kTsel ? z[i] : z[i] - tv[i];
          // Z is never -0 (its sum starts from the bias plus +0, and a sum
          // of +0 and -0 is +0), so d is never -0: its bits as a signed
          // integer are > 0, 0 or < 0 as d is, and their clamp to [-1, 1]
          // (one v_med3_i32) is the sign of d
          lsum += valid ? fabsf(d) : 0.f;
          int si;
          // d may come straight from a matrix-core result, which a vector
          // instruction may read only some cycles after it is written: the
          // compiler pads its own readers but not an asm statement, so the
          // clamp takes the loss sum (a compiler read of d) as an operand
          // and is issued after it
          asm("v_med3_i32 %0, %1, -1, 1" : "=v"(si) : "v"(__float_as_uint(d)), "v"(lsum));
          if (!kFull) si = valid ? si : 0;
          db[nt] += si;
          // -1, 0, 1 as FP32: the high half is the same value in BF16 (the
          // store of that half alone is one ds_write_b16_d16_hi)
          sb[i] = __float_as_uint((float)si);
          rP[w][(pl + i) * kRP + rp_col(pl + i, 16 * nt + r16)] = (unsigned short)(sb[i] >> 16);
        }
        uint2 packed;
        packed.x = __builtin_amdgcn_perm(sb[1], sb[0], 0x07060302u);
        packed.y = __builtin_amdgcn_perm(sb[3], sb[2], 0x07060302u);
        *(uint2*)(&rC[w][(16 * nt + r16) * kRC + pl]) = packed;
      }
    }
    };
    if (lim == kChunk) signs(std::true_type());
    else signs(std::false_type());
    if (ck + kDecPF < ck1) fetch(ck + kDecPF, cur, frc);
    // (3) dW^T += F R^T over the chunk's 32 pixels (A = F hi/lo, B = signs)
    {
      const bf16x8_t fh = as_bf16x8(*(const u16x8*)(fTc + r16 * kFT + 8 * q4));
      const bf16x8_t fl = as_bf16x8(*(const u16x8*)(fTc + 16 * kFT + r16 * kFT + 8 * q4));
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const bf16x8_t rb = as_bf16x8(*(const u16x8*)(&rC[w][(16 * nt + r16) * kRC + 8 * q4]));
        dw[nt] = mfma(fh, rb, dw[nt]);
        dw[nt] = mfma(fl, rb, dw[nt]);
      }
    }
    // (4) this wave's share of dF = W^T R (A = W^T hi/lo, B = signs [channel][pixel])
    f32x4 dfa[2];
#pragma unroll
    for (int cg = 0; cg < 2; ++cg) {
      dfa[cg] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const bf16x8_t rb =
            as_bf16x8(*(const u16x8*)(&rP[w][(16 * cg + r16) * kRP + rp_col(16 * cg + r16, 32 * ks + 8 * q4)]));
        dfa[cg] = mfma(wt_h[ks], rb, dfa[cg]);
        dfa[cg] = mfma(wt_l[ks], rb, dfa[cg]);
      }
    }
#pragma unroll
    for (int cg = 0; cg < 2; ++cg)
#pragma unroll
      for (int i = 0; i < 4; ++i) dfr[par][(w * 16 + 4 * q4 + i) * kChunk + 16 * cg + r16] = dfa[cg][i];
  };
#pragma unroll
  for (int d = 0; d < kDecPF; ++d)
    if (ck0 + d < ck1) fetch(ck0 + d, tr[d], fr[d]);
  for (int64_t cb = ck0; cb < ck1; cb += kDecPF) {
#pragma unroll
    for (int d = 0; d < kDecPF; ++d)
      if (cb + d < ck1) chunk(cb + d, tr[d], fr[d]);
  }
  lds_barrier();
  if (ck1 > ck0) store_df(ck1 - 1, (int)((ck1 - 1 - ck0) & 1));

  // partials of this work-group, times its view's loss scale: dW [C][16],
  // db [C], loss
  float* pb = part + (size_t)blockIdx.x * a.part_stride;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) pb[(size_t)(c0 + 16 * nt + r16) * 16 + 4 * q4 + i] = scale * dw[nt][i];
    int s = db[nt];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (q4 == 0) pb[(size_t)a.C * 16 + c0 + 16 * nt + r16] = scale * (float)s;
  }
  lsum *= scale;
  for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
  if (lane == 0) red[w] = lsum;
  __syncthreads();
  if (t == 0) {
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < kDecWaves; ++u) s += red[u];
    pb[(size_t)a.C * 17] = s;
  }
}

// dW, db and the loss: partials of every work-group added in a fixed order
// (64 outputs per work-group; kRedGroups threads per output take every
// kRedGroups-th partial, so a thread has at most ceil(n_parts / kRedGroups)
// independent loads in flight, then their FP64 sums are added in a fixed
// order).
constexpr int kRedGroups = 16;
__global__ __launch_bounds__(64 * kRedGroups) void k_decoder_reduce(DecArgs a, const float* __restrict__ part,
                                                                   int n_parts) {
  __shared__ double red[kRedGroups][64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + o;
  const int64_t m = (int64_t)a.C * 17 + 1;
  // the partials of up to kRedBatch work-groups per thread are requested
  // before the first is added (n_parts <= kRedGroups kRedBatch in one pass)
  double s = 0.0;
  if (i < m) {
    constexpr int kRedBatch = 16;
    for (int b0 = g; b0 < n_parts; b0 += kRedGroups * kRedBatch) {
      float v[kRedBatch];
#pragma unroll
      for (int u = 0; u < kRedBatch; ++u) {
        const int b = b0 + u * kRedGroups;
        v[u] = b < n_parts ? part[(size_t)b * a.part_stride + i] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < kRedBatch; ++u) s += (double)v[u];
    }
  }
  red[g][o] = s;
  __syncthreads();
  if (g != 0 || i >= m) return;
  s = 0.0;
#pragma unroll
  for (int u = 0; u < kRedGroups; ++u) s += red[u][o];
  if (i < (int64_t)a.C * 16) {
    a.grad_weight[i] = (float)s;
  } else if (i < (int64_t)a.C * 17) {
    a.grad_bias[i - (int64_t)a.C * 16] = (float)s;
  } else if (a.loss) {
    *a.loss = (float)s;
  }
}

template <typename TT>
void launch_t(const DecArgs& a, float* part, int grid, hipStream_t s) {
  if (a.C == 256)
    hipLaunchKernelGGL((k_decoder<TT, 2, 8>), dim3(grid), dim3(64 * 8), 0, s, a, part);
  else
    hipLaunchKernelGGL((k_decoder<TT, 2, 16>), dim3(grid), dim3(64 * 16), 0, s, a, part);
}

}  // namespace

bool decoder_dim_ok(int C) { return C == 256 || C == 512; }

int decoder_assign(DecArgs& a, int cap) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int budget = cus < cap ? cus : cap;   // one 8-wave work-group per CU
  int64_t ch[kDecMaxViews];
  int g[kDecMaxViews], total = 0;
  for (int v = 0; v < a.n_views; ++v) {
    ch[v] = (a.v[v].n + kChunk - 1) / kChunk;
    g[v] = 1;
    ++total;
  }
  // each further work-group goes to the view whose work-groups have the
  // most chunks each (the first such view), while it has chunks to spare
  while (total < budget) {
    int best = -1;
    int64_t most = 0;
    for (int v = 0; v < a.n_views; ++v) {
      const int64_t per = (ch[v] + g[v] - 1) / g[v];
      if (g[v] < ch[v] && per > most) {
        most = per;
        best = v;
      }
    }
    if (best < 0) break;
    ++g[best];
    ++total;
  }
  int g0 = 0;
  for (int v = 0; v < a.n_views; ++v) {
    a.v[v].g0 = g0;
    a.v[v].groups = g[v];
    g0 += g[v];
  }
  return g0;
}

void launch_decoder(const DecArgs& a, int target_bf16, float* part, int grid, hipStream_t s) {
  if (target_bf16) launch_t<unsigned short>(a, part, grid, s);
  else launch_t<float>(a, part, grid, s);
  const int64_t m = (int64_t)a.C * 17 + 1;
  hipLaunchKernelGGL(k_decoder_reduce, dim3((unsigned)((m + 63) / 64)), dim3(64 * kRedGroups), 0, s, a, part,
                     grid);
}

}  // namespace lgs

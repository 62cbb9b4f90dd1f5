// Per-pixel compositing of RGB + depth + 16-d feature (forward) and its
// reverse-order backward, plus the per-Gaussian segmented reduction of the
// backward's partial sums.
//
// Paper: Sec. III-B.1 renders the image and the feature map with the usual
// 3D Gaussian Splatting rasterizer; Eq. (1) uses the rendered depth; Sec. III-B.3
// optimises the Gaussians through this renderer.  Per pixel, front to back
// over the Gaussians of its tile in (depth, index) order:
//   alpha = min(alpha_max, o exp(-m2/2)), skipped unless m2 <= cutoff2 and
//   alpha >= alpha_min; T' = T (1 - alpha); stop before T' < T_eps;
//   Y += alpha T [r, g, b, z, f0..f15]; T = T'.
//
// Execution.  One wave64 renders one 8x8 pixel block (one pixel per lane)
// and walks the list of the binning tile that holds the block, 64 entries at
// a time: each lane loads one entry's geometry record with a vector load and
// tests whether the entry's ellipse can reach the block at all (cull_hit); a
// ballot gives the mask of entries to evaluate.  The wave then visits those
// entries in list order.  What an entry carries is wave-uniform: its fields
// are broadcast to SGPRs (v_readlane from the lane that loaded it, or a
// scalar load) and used directly as VALU operands, so no LDS staging and no
// per-lane gathers are needed.  The wave leaves the list as soon as a ballot
// shows every lane finished.  Waves pop blocks from per-XCD work queues
// (persistent grid).
//
// Backward.  Each wave restarts from the last contributor of its pixels and
// walks the list backwards, recovering T before each entry as T / (1 - alpha)
// and the weighted sum of what lies behind as a single running scalar.  Per
// entry, the 6 geometric sums (the moments of dL/dm2 over the pixel offsets
// dx, dy, dx^2, dx dy, dy^2, and dL/dalpha-weighted G for the opacity) are
// summed over the wave by a butterfly transpose-reduction; the 20 colour /
// depth / feature partials, sum_p w_p g_p, are collected for batches of 8
// entries as a (entries x pixels) x (pixels x channels) product on the matrix
// cores.  Both go to the entry's own (Gaussian, block) slot; a segmented
// reduction over each Gaussian's slots then forms its gradient.  No atomics:
// results are deterministic run to run.
#include "lgs_internal.h"

#include <type_traits>

namespace lgs {
namespace {

// The forward and the backward evaluate an entry with this one function so
// that their discrete decisions agree bit for bit.
struct Eval {
  float m2, G, araw, alpha;
  bool pass;
};

__device__ __forceinline__ Eval eval_entry(float dx, float dy, float qa, float qb2, float qc, float o,
                                           float cutoff2, float alpha_max, float alpha_min) {
#pragma clang fp contract(off)
  Eval e;
  const float t1 = qc * dy;
  const float t2 = t1 * dy;
  const float t3 = qb2 * dx;
  const float t4 = __builtin_fmaf(t3, dy, t2);
  const float t5 = qa * dx;
  e.m2 = __builtin_fmaf(t5, dx, t4);
  e.G = __builtin_amdgcn_exp2f(e.m2 * -0.72134752044448170f);   // exp(-m2/2)
  e.araw = o * e.G;
  // min(araw, alpha_max) as a single v_min_f32 (equal to fminf here: araw
  // is a product, never a signalling NaN); fminf would first canonicalise
  // the setting with an instruction of its own at every entry
  asm("v_min_f32 %0, %1, %2" : "=v"(e.alpha) : "s"(alpha_max), "v"(e.araw));
  e.pass = (e.m2 <= cutoff2) && (e.alpha >= alpha_min);
  return e;
}

__device__ __forceinline__ bool block_in_bbox(uint32_t bb, uint32_t bx, uint32_t by) {
  return bx >= (bb & 255u) && bx <= ((bb >> 8) & 255u) && by >= ((bb >> 16) & 255u) && by <= (bb >> 24);
}

// Can the entry's ellipse reach the 8x8 block (bx, by) at all?  The minimum
// of the quadratic form over the block's pixel rectangle is 0 when the
// rectangle holds the centre, else the smallest of the four edge minima (a
// clamped 1-D minimiser per edge).  The entry is skipped only when that
// minimum exceeds the per-pixel cut min(cutoff2, 2 ln(o / alpha_min)) by a
// margin that covers the FP32 rounding of both this test and the per-pixel
// evaluation (whose error grows with (qa + qc) |d|^2), so the test never
// drops an entry that eval_entry would accept at some pixel of the block.
// The edge minimisers use the hardware reciprocal (about 1 ulp): a minimiser
// off by that much raises the edge minimum by a second-order amount, far
// inside the margin.
__device__ __forceinline__ bool cull_hit(const GeomRec& g, uint32_t bx, uint32_t by, float cutoff2,
                                         float log2_alpha_min) {
  const int bx0 = (int)(g.bbox & 255u), by0 = (int)((g.bbox >> 16) & 255u);
  const float x0 = (float)(8 * ((int)bx - bx0)) - g.mx, x1 = x0 + 7.f;
  const float y0 = (float)(8 * ((int)by - by0)) - g.my, y1 = y0 + 7.f;
  float m = 0.f;
  if (!(x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f)) {
    const float ia = -g.qb2 * __builtin_amdgcn_rcpf(2.f * g.qa), ic = -g.qb2 * __builtin_amdgcn_rcpf(2.f * g.qc);
    auto qf = [&](float dx, float dy) { return g.qa * dx * dx + g.qb2 * dx * dy + g.qc * dy * dy; };
    // clamps as one v_med3_f32 each (finite operands: no NaN handling)
    const float e0 = qf(x0, __builtin_amdgcn_fmed3f(ic * x0, y0, y1));
    const float e1 = qf(x1, __builtin_amdgcn_fmed3f(ic * x1, y0, y1));
    const float e2 = qf(__builtin_amdgcn_fmed3f(ia * y0, x0, x1), y0);
    const float e3 = qf(__builtin_amdgcn_fmed3f(ia * y1, x0, x1), y1);
    m = __builtin_fminf(__builtin_fminf(e0, e1), __builtin_fminf(e2, e3));
  }
  const float r2 = fminf(cutoff2, 1.3862943611198906f * (__builtin_amdgcn_logf(g.o) - log2_alpha_min));
  const float d2 = fmaxf(x0 * x0, x1 * x1) + fmaxf(y0 * y0, y1 * y1);
  return m <= r2 * 1.0001f + 1e-3f + 4e-6f * (g.qa + g.qc) * d2;
}

// A list entry's whole record for the cull test, requested as one: its
// fields are used at once, so the compiler cannot defer those the box test
// does not need below that test's branch (a further dependent round trip
// per chunk).
__device__ __forceinline__ GeomRec load_rec_whole(const GeomRec* __restrict__ p) {
  const GeomRec g = *p;
  asm volatile("" ::"v"(g.mx), "v"(g.my), "v"(g.qa), "v"(g.qb2), "v"(g.qc), "v"(g.o), "v"(g.z), "v"(g.bbox));
  return g;
}

// Record of list entry j's Gaussian (rid in lane j) by a scalar load whose
// offset is a 32-bit register (records sit below 2^32 bytes): one shift of
// the index instead of 64-bit address arithmetic per entry.
__device__ __forceinline__ GeomRec rec_of_lane(const GeomRec* __restrict__ geom, uint32_t rid_l, uint32_t j) {
  const uint32_t off = (uint32_t)__builtin_amdgcn_readlane((int)rid_l, (int)j) << 5;
  return *(const GeomRec*)((const char*)geom + off);
}

__device__ __forceinline__ float bcast(float x, uint32_t j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
}

// Appearance record words of Gaussian g (10 words in BF16 storage, 20 in
// FP32) and their unpacking into the 20-vector [r, g, b, (z), f0..f15]; slot
// 3 is filled by the caller with the view's depth.
template <bool BF16>
__device__ __forceinline__ void load_app_words(const void* __restrict__ app, uint32_t g, uint32_t w[20]) {
  // (a 32-bit byte offset: the records stay below 2^32 bytes)
  const uint32_t* a = (const uint32_t*)((const char*)app + g * (BF16 ? 40u : 80u));
#pragma unroll
  for (int k = 0; k < (BF16 ? 10 : 20); ++k) w[k] = a[k];
}

template <bool BF16>
__device__ __forceinline__ void y_from_words(const uint32_t u[20], float y[20]) {
  if (BF16) {
    y[0] = __uint_as_float(u[0] << 16);
    y[1] = __uint_as_float(u[0] & 0xffff0000u);
    y[2] = __uint_as_float(u[1] << 16);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      y[4 + 2 * k] = __uint_as_float(u[2 + k] << 16);
      y[5 + 2 * k] = __uint_as_float(u[2 + k] & 0xffff0000u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 20; ++k) y[k] = __uint_as_float(u[k]);
  }
}

// Pop one work item for the whole wave.  Every active lane executes the
// atomic (no lane-dependent branch around it): the first active lane adds 1,
// the others 0, and the first active lane's return value is broadcast.  A
// "lane 0 only" branch here let the compiler merge it with the other
// lane-0 branches of the loop and drop lane 0 from EXEC at the back edge,
// after which readfirstlane read another lane's stale value.
__device__ __forceinline__ uint32_t pop_item(uint32_t* counter) {
  const uint64_t exec = __builtin_amdgcn_read_exec();
  const uint32_t lane = __lane_id();
  const bool leader = lane == (uint32_t)(__builtin_ctzll(exec));
  const uint32_t old = atomicAdd(counter, leader ? 1u : 0u);
  return __builtin_amdgcn_readfirstlane(old);
}

// Next work item of the calling wave from the queue of its XCD (workgroup
// index mod kQueues), or n_items once that queue is empty.  Wave-uniform.
// (Taking items from other queues once the own queue is empty was measured
// slower: the longest-first order already leaves a short tail.)
__device__ __forceinline__ uint32_t next_item(uint32_t* ctr, const uint32_t* __restrict__ qoff, uint32_t q,
                                              uint32_t n_items) {
  const uint32_t k = pop_item(&ctr[q * kLineWords]);
  const uint32_t b = qoff[q], e = qoff[q + 1];
  return k < e - b ? b + k : n_items;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Forward accumulation on the matrix cores (BF16 appearance).  The 20 sums
// acc[p][s] = sum_e w[p][e] y[e][s] of a batch of 8 entries form one
// v_mfma_f32_16x16x32_bf16 per group of 4 channel slots s and per term of
// the weights: the K index runs over (pixel group g' = lane / 16, entry e),
// the weights w (the B operand) are each lane's own, and the A operand is
// block diagonal (the appearance y in the rows of the lane's own pixel group,
// zero elsewhere), so the result lands in the lane of its pixel: lane l holds
// acc[l][4 j + i] in register i of block j.  The weights are split exactly
// into three BF16 terms (8 significant bits each) and the BF16 appearance is
// exact, so every product is exact and only the FP32 accumulation rounds.
// The depth slot is accumulated separately in FP32.
// LDS of one wave: the batch's appearance [20 slots][8 entries] in rows 0-19
// of a [64][8] area (lane l stores into row l, so the per-entry store needs
// no lane mask; rows 20-63 are never read), a zero block [20][8], and the
// weights [3 terms][64 pixels][8 entries] (BF16).
constexpr int kFwdY = 20 * 8;
constexpr int kFwdYRows = 64 * 8;
constexpr int kFwdW = 64 * 8;
constexpr int kFwdWaveLds = (kFwdYRows + kFwdY + 3 * kFwdW) * 2;

// FP32 appearance: eight waves per SIMD (64 VGPRs), measured faster than the
// compiler's own register choice, which leaves room for only seven.  BF16
// appearance: seven (72 VGPRs), so that a batch's weight operands stay in
// registers across its five channel blocks (faster than eight waves that
// re-read them).
// NC: per-pixel contributor counts are written (a caller asked for them);
// without them the entry loop keeps no count.
template <bool BF16, bool CNT, bool NC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BF16 ? 7 : 8, BF16 ? 7 : 8))) k_raster_fwd(
    Settings st, const ViewDesc* __restrict__ views, const ViewImages* __restrict__ out,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ vals,
    const GeomRec* __restrict__ geom, const void* __restrict__ app, uint32_t npad_mask,
    const uint32_t* __restrict__ items, const uint32_t* __restrict__ qoff, uint32_t n_items,
    Counters* __restrict__ cnt, int32_t* __restrict__ last_idx, float* __restrict__ T_state) {
  const int lane = threadIdx.x & 63;
  if (cnt->overflow) return;
  extern __shared__ unsigned short lds_f[];
  unsigned short* ys = lds_f + (threadIdx.x >> 6) * (kFwdWaveLds / 2);
  unsigned short* yz = ys + kFwdYRows;
  unsigned short* ws = yz + kFwdY;
  // A-operand rows: lane l reads slot 4 j + (l & 3) when its row group
  // (l & 15) / 4 equals its k-block l / 16, else the zero block
  const unsigned short* abase = (((lane & 15) >> 2) == (lane >> 4) ? ys : yz) + (lane & 3) * 8;
  // the appearance slot this lane loads per entry (lanes past the 20 slots
  // repeat the last one, into rows no product reads); the records' byte
  // offsets stay below 2^32, so each load takes a 32-bit lane offset
  const uint32_t ylane = lane < 20 ? (uint32_t)lane : 19u;
  const unsigned short* __restrict__ app16 = (const unsigned short*)app;
  if (BF16) {
    // the zero block, and the weights: a partial batch leaves the weights of
    // its unused entries as they were (their appearance is zeroed instead),
    // so they must never hold a NaN or infinity from whatever LDS held before
    ((uint32_t*)yz)[lane] = 0u;
    if (lane < kFwdY / 2 - 64) ((uint32_t*)yz)[64 + lane] = 0u;
#pragma unroll
    for (int t = 0; t < 3; ++t) *(uint4*)(ws + t * kFwdW + lane * 8) = make_uint4(0u, 0u, 0u, 0u);
  }
  // this wave's work (CNT: the profiling variant), added to the 64-bit
  // counters once at the end (a wave's own count stays far below 2^32); the
  // timed variant carries none of this bookkeeping in its entry loop
  uint32_t n_eval = 0, n_con = 0, n_ent = 0;
  const uint32_t q = blockIdx.x % (uint32_t)kQueues;
  for (;;) {
    const uint32_t it = next_item(cnt->work_q, qoff, q, n_items);
    if (it >= n_items) break;
    const uint32_t item = items[it];
    const uint32_t bx = item & 255u, by = (item >> 8) & 255u, v = item >> 16;
    const ViewDesc* V = views + v;
    const int W = V->W, H = V->H;
    const int px = (int)bx * kBlock + (lane & 7), py = (int)by * kBlock + (lane >> 3);
    const bool inside = px < W && py < H;
    const uint32_t tile = (uint32_t)V->tile_off + (by >> st.tile_shift) * (uint32_t)V->tiles_x +
                          (bx >> st.tile_shift);
    const uint2 r = ranges[tile];
    float T = 1.f;
    float acc[20];   // FP32 appearance
#pragma unroll
    for (int c = 0; c < 20; ++c) acc[c] = 0.f;
    f32x4 D[5];      // BF16 appearance: slots 4 j .. 4 j + 3 of this lane's pixel
#pragma unroll
    for (int jb = 0; jb < 5; ++jb) D[jb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float accz = 0.f;
    int nb = 0;
    auto flush = [&]() {
      if (nb < 8 && lane < 20)
        for (int e = nb; e < 8; ++e) ys[lane * 8 + e] = 0;
      // the three weight terms (B) are the same for the five channel
      // blocks: read once, 8 LDS reads per batch instead of 20 (12 more
      // VGPRs, hence 7 waves per SIMD instead of 8)
      bf16x8_t bw[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) bw[t] = *(const bf16x8_t*)(ws + t * kFwdW + lane * 8);
#pragma unroll
      for (int jb = 0; jb < 5; ++jb) {
        const bf16x8_t a = *(const bf16x8_t*)(abase + 32 * jb);
#pragma unroll
        for (int t = 0; t < 3; ++t) D[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t], D[jb], 0, 0, 0);
      }
      nb = 0;
    };
    int32_t last = -1, ncon = 0;
    // the lanes still compositing, as a wave mask in SGPRs: per-lane tests
    // enter it through ballots of single comparisons and leave it through
    // inverse ballots, so the bookkeeping costs scalar instructions only
    uint64_t live = __builtin_amdgcn_ballot_w64(inside);
    bool finished = live == 0ull;
    // the list entries of the next chunk are requested a chunk ahead
    uint32_t rid_n = 0;
    if (r.x + (uint32_t)lane < r.y) rid_n = vals[r.x + (uint32_t)lane];
    for (uint32_t base = r.x; base < r.y && !finished; base += 64) {
      // lane l takes entry base + l and decides whether the wave visits it
      const uint32_t kl = base + (uint32_t)lane;
      const uint32_t rid_l = rid_n;
      GeomRec g_l{};
      bool hit = false;
      if (kl < r.y) {
        g_l = load_rec_whole(geom + rid_l);
        hit = block_in_bbox(g_l.bbox, bx, by) && cull_hit(g_l, bx, by, st.cutoff2, st.log2_alpha_min);
      }
      if (kl + 64u < r.y) rid_n = vals[kl + 64u];
      uint64_t hm = __builtin_amdgcn_ballot_w64(hit);
      // the appearance of the entry to visit next is requested at the end of
      // the current one, so its latency overlaps that entry's evaluation
      uint32_t j = hm ? (uint32_t)__builtin_ctzll(hm) : 0u;
      uint32_t aw[20];
      unsigned short yh = 0;   // BF16: this lane's channel slot of the entry's appearance
      // the next entry's geometry: with BF16 appearance a scalar load issued
      // one entry ahead (the appearance goes through vector loads, so the
      // SGPRs are free for it); with FP32 appearance (20 scalar appearance
      // words) broadcast from the lane that loaded it
      GeomRec gn{};
      if (hm) {
        if (BF16) gn = rec_of_lane(geom, rid_l, j);
        const uint32_t g0 = __builtin_amdgcn_readlane(rid_l, j) & npad_mask;
        if (BF16) {
          yh = *(const unsigned short*)((const char*)app16 + (g0 * 40u + 2u * ylane));
        } else {
          load_app_words<BF16>(app, g0, aw);
        }
      }
      while (hm) {
        hm &= hm - 1ull;
        GeomRec gr;
        if (BF16) {
          gr = gn;
        } else {
          gr.mx = bcast(g_l.mx, j);
          gr.my = bcast(g_l.my, j);
          gr.qa = bcast(g_l.qa, j);
          gr.qb2 = bcast(g_l.qb2, j);
          gr.qc = bcast(g_l.qc, j);
          gr.o = bcast(g_l.o, j);
          gr.z = bcast(g_l.z, j);
          gr.bbox = __builtin_amdgcn_readlane(g_l.bbox, j);
        }
        const uint32_t bb = gr.bbox;
        if (CNT) {
          n_eval += (uint32_t)__popcll(live);
          ++n_ent;
        }
        const float dx = (float)(px - 8 * (int)(bb & 255u)) - gr.mx;
        const float dy = (float)(py - 8 * (int)((bb >> 16) & 255u)) - gr.my;
        const Eval e = eval_entry(dx, dy, gr.qa, gr.qb2, gr.qc, gr.o, st.cutoff2, st.alpha_max, st.alpha_min);
        const float Tn = T * (1.f - e.alpha);
        // e.pass, as a mask
        const uint64_t pm = live & __builtin_amdgcn_ballot_w64(e.m2 <= st.cutoff2) &
                            __builtin_amdgcn_ballot_w64(e.alpha >= st.alpha_min);
        const uint64_t tm = pm & __builtin_amdgcn_ballot_w64(Tn < st.T_eps);   // terminates here
        live &= ~tm;
        const uint64_t cmask = pm & ~tm;
        if (cmask != 0ull) {
          const bool con = __builtin_amdgcn_inverse_ballot_w64(cmask);
          if (CNT) n_con += (uint32_t)__popcll(cmask);
          const float w = con ? e.alpha * T : 0.f;
          if (BF16) {
            accz = __builtin_fmaf(w, gr.z, accz);
            // w = hi + mid + lo exactly: each term keeps the top 8 significant
            // bits of what is left (truncation), so each is a BF16 value
            const float whi = __uint_as_float(__float_as_uint(w) & 0xffff0000u);
            const float r1 = w - whi;
            const float wmid = __uint_as_float(__float_as_uint(r1) & 0xffff0000u);
            const float wlo = r1 - wmid;
            ws[lane * 8 + nb] = (unsigned short)(__float_as_uint(whi) >> 16);
            ws[kFwdW + lane * 8 + nb] = (unsigned short)(__float_as_uint(wmid) >> 16);
            ws[2 * kFwdW + lane * 8 + nb] = (unsigned short)(__float_as_uint(wlo) >> 16);
            ys[lane * 8 + nb] = yh;
          } else {
            float y[20];
            y_from_words<BF16>(aw, y);
            y[3] = gr.z;
#pragma unroll
            for (int c = 0; c < 20; ++c) acc[c] = __builtin_fmaf(w, y[c], acc[c]);
          }
          T = con ? Tn : T;
          last = con ? (int32_t)(base + j) : last;
          if (NC) ncon += con ? 1 : 0;
          if (BF16 && ++nb == 8) flush();
        }
        if (live == 0ull) {
          finished = true;
          break;
        }
        if (hm) {
          j = (uint32_t)__builtin_ctzll(hm);
          if (BF16) gn = rec_of_lane(geom, rid_l, j);
          const uint32_t g0 = __builtin_amdgcn_readlane(rid_l, j) & npad_mask;
          if (BF16) {
            yh = *(const unsigned short*)((const char*)app16 + (g0 * 40u + 2u * ylane));
          } else {
            load_app_words<BF16>(app, g0, aw);
          }
        }
      }
    }
    if (BF16) {
      if (nb > 0) flush();
#pragma unroll
      for (int jb = 0; jb < 5; ++jb)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[4 * jb + i] = D[jb][i];
      acc[3] = accz;
    }
    if (inside) {
      const ViewImages o = out[v];
      const size_t HW = (size_t)W * H, p = (size_t)py * W + px;
#pragma unroll
      for (int c = 0; c < 3; ++c) o.rgb[c * HW + p] = acc[c];
      o.depth[p] = acc[3];
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < st.nfeat) o.feat[c * HW + p] = acc[4 + c];
      o.T[p] = T;
      if (NC && o.n_contrib) o.n_contrib[p] = ncon;
      last_idx[(size_t)V->pix_off + p] = last;
      T_state[(size_t)V->pix_off + p] = T;
    }
  }
  if (CNT && lane == 0) {
    atomicAdd(&cnt->fwd_evals, (unsigned long long)n_eval);
    atomicAdd(&cnt->fwd_contrib, (unsigned long long)n_con);
    atomicAdd(&cnt->fwd_entries, (unsigned long long)n_ent);
  }
}

// Butterfly transpose-reductions: every lane holds a vector of values and
// the lanes' vectors are summed value by value, each lane ending with one of
// the sums.  Each step pairs every lane with a partner, each keeps one half
// of its values and adds the partner's copy of that half: cross-row steps use
// the gfx950 permlane swaps (no selects: the swap itself hands each half to
// the lane that keeps it), in-row steps a bit-select and a DPP read of the
// partner.
__device__ __forceinline__ float bsel(bool hi, float a, float b) {   // hi ? b : a
  const uint32_t m = hi ? 0xffffffffu : 0u;
  return __uint_as_float((__float_as_uint(a) & ~m) | (__float_as_uint(b) & m));
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ int wave_max_i32(int x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, __shfl_xor(x, off, 64));
  return x;
}

constexpr int kZRow = 72;                  // bf16 per LDS row (64 pixels + pad; 144 B, 16-B aligned)
// Blend-weight rows of a batch of 8 entries: three exact BF16 terms each.
constexpr int kWRows = 24;
// At each flush the batch's partial records are assembled in the weight
// rows, whose weights the products have consumed by then: record e (36
// floats: the 32 of a slot + pad) fills the 144 bytes of weight row e.  The
// geometric sums of the batch's entries wait in a small area of their own.
constexpr int kRecLds = 36;
static_assert(kRecLds * 4 == kZRow * 2, "a record fills one weight row");
constexpr int kGeoStride = 8;              // floats per entry of the geometric staging
constexpr int kGeoBytes = 8 * kGeoStride * 4;
// LDS bytes of one backward wave: upstream rows, blend-weight rows,
// geometric staging
__host__ __device__ constexpr int bwd_wave_lds_bytes(int up_mode) {
  return (bwd_upstream_rows(up_mode) + kWRows) * kZRow * 2 + kGeoBytes;
}
// FP32 -> BF16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

// Transpose-reduction of 6 values over the whole wave: on exit lane l holds
// the wave sum of value red6_index(l).  Partners: l ^ 32 (permlane32 swap:
// lanes below 32 keep values 0..2, the others 3..5), l ^ 16 (permlane16
// swap: values 0 / 1 split by row parity, value 2 summed in every row), l ^ 8
// (row_ror:8: bit 3 chooses between the two), then 7 - (l & 7), l ^ 2, l ^ 1.
__device__ __forceinline__ int red6_index(int l) { return 3 * (l >> 5) + ((l & 8) ? 2 : (l >> 4) & 1); }
__device__ __forceinline__ float transpose_reduce6(const float v[6], int lane) {
  float a[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[3 + i]), false, false);
    a[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  auto r01 = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[0]), __float_as_uint(a[1]), false, false);
  const float b = __uint_as_float(r01[0]) + __uint_as_float(r01[1]);
  auto r22 = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[2]), __float_as_uint(a[2]), false, false);
  const float b2 = __uint_as_float(r22[0]) + __uint_as_float(r22[1]);
  const bool h8 = (lane & 8) != 0;
  float c = bsel(h8, b, b2) + dpp<0x128>(bsel(h8, b2, b));
  c = c + dpp<0x141>(c);
  c = c + dpp<0x4E>(c);
  return c + dpp<0xB1>(c);
}

// Waves per SIMD: what the LDS of each upstream form allows (six for the
// fused L1 gradient, 80 VGPRs, measured fastest; five with the colour
// gradient's extra rows; four with a given upstream's hi + lo rows), so that
// the VGPR budget is no tighter than the occupancy LDS permits.
constexpr int bwd_waves_per_eu(int up_mode) { return up_mode == UP_L1 ? 6 : (up_mode == UP_RGB ? 5 : 4); }
template <bool BF16, int UPM, bool CNT>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(bwd_waves_per_eu(UPM), bwd_waves_per_eu(UPM)))) k_raster_bwd(
    Settings st, const ViewDesc* __restrict__ views, const ViewImages* __restrict__ upstream,
    const ViewImages* __restrict__ fwd_out, const ViewImages* __restrict__ targets,
    const float* __restrict__ loss_w, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ vals, const GeomRec* __restrict__ geom,
    const void* __restrict__ app, uint32_t npad_mask, const uint32_t* __restrict__ items,
    const uint32_t* __restrict__ qoff, uint32_t n_items, Counters* __restrict__ cnt,
    const int32_t* __restrict__ last_idx,
    const float* __restrict__ T_state, const uint32_t* __restrict__ slot_base,
    float* __restrict__ partials, uint8_t* __restrict__ mask) {
  const int lane = threadIdx.x & 63;
  extern __shared__ unsigned short lds_z[];
  // upstream per channel: the sign of the L1 residual (formed here from the
  // forward's images and the targets; exact in BF16, the per-channel scale is
  // applied after the product) or a given FP32 value (split hi + lo)
  constexpr bool kSignRGB = UPM == UP_L1;
  constexpr bool kSignDF = UPM != UP_EXPLICIT;
  // this wave's LDS rows (BF16, 64 pixels + pad each): the block's upstream
  // per channel, hi (20) and lo (for the given channels: 20, or the 3 colour
  // channels), and the blend weights of up to 8 batched entries in three
  // exact terms (rows 0-7, 8-15, 16-23); then the geometric staging
  constexpr int kGRows = bwd_upstream_rows(UPM);
  unsigned short* lz = lds_z + (threadIdx.x >> 6) * (bwd_wave_lds_bytes(UPM) / 2);
  unsigned short* wz = lz + kGRows * kZRow;
  float* recs = (float*)wz;                         // records, at flush time
  float* geo = (float*)(wz + kWRows * kZRow);       // 8 entries x kGeoStride floats
  const int grp = lane >> 4, col = lane & 15;
  if (cnt->overflow) return;
  // this wave's work (CNT: the profiling variant), added to the 64-bit
  // counters once at the end (a wave's own count stays far below 2^32)
  uint32_t n_eval = 0, n_con = 0, n_ent = 0, n_wr = 0;
  const uint32_t q = blockIdx.x % (uint32_t)kQueues;
  for (;;) {
    const uint32_t it = next_item(cnt->work_qb, qoff, q, n_items);
    if (it >= n_items) break;
    const uint32_t item = items[it];
    const uint32_t bx = item & 255u, by = (item >> 8) & 255u, v = item >> 16;
    const ViewDesc* V = views + v;
    const int W = V->W, H = V->H;
    const int px = (int)bx * kBlock + (lane & 7), py = (int)by * kBlock + (lane >> 3);
    const bool inside = px < W && py < H;
    const size_t HW = (size_t)W * H, p = (size_t)py * W + px;
    int32_t last = -1;
    float Tfin = 1.f, gT = 0.f;
    float g[20];
#pragma unroll
    for (int c = 0; c < 20; ++c) g[c] = 0.f;
    if (inside) {
      last = last_idx[(size_t)V->pix_off + p];
      Tfin = T_state[(size_t)V->pix_off + p];
      if (kSignDF) {
        const ViewImages Y = fwd_out[v], Yt = targets[v];
        const float s_rgb = loss_w[0] / (3.f * (float)HW), s_d = loss_w[1] / (float)HW;
        const float s_f = loss_w[2] / (16.f * (float)HW);
        if (kSignRGB) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float d = Y.rgb[c * HW + p] - Yt.rgb[c * HW + p];
            g[c] = d > 0.f ? s_rgb : (d < 0.f ? -s_rgb : 0.f);
          }
        } else {
          const float* __restrict__ Urgb = upstream[v].rgb;
#pragma unroll
          for (int c = 0; c < 3; ++c) g[c] = Urgb[c * HW + p];
        }
        {
          const float d = Y.depth[p] - Yt.depth[p];
          g[3] = d > 0.f ? s_d : (d < 0.f ? -s_d : 0.f);
        }
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const float d = c < st.nfeat ? Y.feat[c * HW + p] - Yt.feat[c * HW + p] : 0.f;
          g[4 + c] = d > 0.f ? s_f : (d < 0.f ? -s_f : 0.f);
        }
      } else {
        const ViewImages U = upstream[v];
#pragma unroll
        for (int c = 0; c < 3; ++c) g[c] = U.rgb[c * HW + p];
        g[3] = U.depth[p];
#pragma unroll
        for (int c = 0; c < 16; ++c) g[4 + c] = c < st.nfeat ? U.feat[c * HW + p] : 0.f;
        if (U.T) gT = U.T[p];
      }
    }
    // every lane holds the same maximum; readfirstlane makes that visible to
    // the compiler, so the entry loop below stays on the scalar unit
    const int kmax = __builtin_amdgcn_readfirstlane(wave_max_i32(last));
    if (kmax < 0) continue;
    const uint32_t tile = (uint32_t)V->tile_off + (by >> st.tile_shift) * (uint32_t)V->tiles_x +
                          (bx >> st.tile_shift);
    const uint32_t kbeg = ranges[tile].x;
    const float gTT = gT * Tfin;
    float Tc = Tfin, sB = 0.f;
    // upstream rows: for the fused L1 gradient the sign (exact in BF16; the
    // per-channel scale is applied to the MFMA result), else hi + lo BF16.
    // The colour partials of a batch of entries, dY[e][c] = sum_p w[p][e] g[p][c],
    // are a (entries x pixels) x (pixels x channels) product: v_mfma_f32_16x16x32_bf16
    // on the two-term splits (hi.hi + lo.hi, + hi.lo for a general upstream),
    // FP32 accumulation.
    float gscale[3] = {1.f, 1.f, 1.f};
    if (kSignDF) {
      const float HWf = (float)HW;
      gscale[0] = kSignRGB ? loss_w[0] / (3.f * HWf) : 1.f;
      gscale[1] = loss_w[1] / HWf;
      gscale[2] = loss_w[2] / (16.f * HWf);
    }
#pragma unroll
    for (int c = 0; c < 20; ++c) {
      if (c < 3 ? kSignRGB : kSignDF) {
        const float sgn = g[c] > 0.f ? 1.f : (g[c] < 0.f ? -1.f : 0.f);
        lz[c * kZRow + lane] = bf16_rne(sgn);
      } else {
        const unsigned short hi = bf16_rne(g[c]);
        lz[c * kZRow + lane] = hi;
        lz[(20 + c) * kZRow + lane] = bf16_rne(g[c] - bf16_to_f(hi));
      }
    }
    // Feature part of gy = sum_c g[c] y[c] with BF16 appearance and the sign
    // upstream: s_f sum_f sign_f y_f, the sum by packed BF16 dot products of
    // the appearance words (two features each, used as they are stored) with
    // the signs packed the same way; every product is exact.
    constexpr bool kDotGy = BF16 && kSignDF;
    uint32_t sg2[8];
    if (kDotGy) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const float a = g[4 + 2 * k], b = g[5 + 2 * k];
        const uint32_t lo = a > 0.f ? 0x3f80u : (a < 0.f ? 0xbf80u : 0u);
        const uint32_t hi = b > 0.f ? 0x3f80u : (b < 0.f ? 0xbf80u : 0u);
        sg2[k] = lo | (hi << 16);
      }
    }
    int nb = 0;
    uint32_t slotv = 0;   // lane e: the slot of the batch's entry e
    // Write the batch's nb partial records: the colour partials, sum_p w_p
    // g_p, come from the matrix cores; the three weight terms go through
    // K-stacked products (each term against the same upstream rows), so
    // with a sign upstream every product is exact and only the FP32
    // accumulation rounds.  Then the records are assembled in the consumed
    // weight rows (colour partials and the staged geometric sums), lanes
    // store 16-byte quarters of them (seven quarters, 112 bytes, of each
    // 128-byte slot; 8 lanes per record) and the first lane of each record
    // sets the slot's mask byte.
    auto flush = [&]() {
      f32x4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
      const int er = col & 7;
      const int ch1 = col < 4 ? 16 + col : 16;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int off = 32 * ks + 8 * grp;
        bf16x8_t aw[3];   // output rows 8..15 repeat rows 0..7
#pragma unroll
        for (int t = 0; t < 3; ++t) aw[t] = *(const bf16x8_t*)(wz + (8 * t + er) * kZRow + off);
        const bf16x8_t bh0 = *(const bf16x8_t*)(lz + col * kZRow + off);
        bf16x8_t bh1 = *(const bf16x8_t*)(lz + ch1 * kZRow + off);
        if (col >= 4) bh1 = (bf16x8_t){};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t], bh0, c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t], bh1, c1, 0, 0, 0);
        }
        if (UPM == UP_EXPLICIT) {
          // the given upstream's lo term (relative 2^-8 of hi) against the two
          // leading weight terms: the dropped products are below 2^-24
          const bf16x8_t bl0 = *(const bf16x8_t*)(lz + (20 + col) * kZRow + off);
          bf16x8_t bl1 = *(const bf16x8_t*)(lz + (20 + ch1) * kZRow + off);
          if (col >= 4) bl1 = (bf16x8_t){};
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t], bl0, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t], bl1, c1, 0, 0, 0);
          }
        } else if (UPM == UP_RGB) {
          // lo rows exist for the three colour channels only
          bf16x8_t bl0 = *(const bf16x8_t*)(lz + (20 + (col < 3 ? col : 0)) * kZRow + off);
          if (col >= 3) bl0 = (bf16x8_t){};
#pragma unroll
          for (int t = 0; t < 2; ++t) c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[t], bl0, c0, 0, 0, 0);
        }
      }
      // every read of the weight rows above precedes the record writes below
      // (LDS operations of a wave run in order; this keeps the compiler from
      // moving the differently typed accesses across each other)
      asm volatile("" ::: "memory");
      const float s0 = col < 3 ? gscale[0] : (col == 3 ? gscale[1] : gscale[2]);
      const float s1 = gscale[2];
      if (grp < 2) {   // output rows 8..15 repeat rows 0..7
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float* rec = recs + (4 * grp + i) * kRecLds;
          rec[6 + col] = c0[i] * s0;
          if (col < 4) rec[22 + col] = c1[i] * s1;
        }
      }
      if (lane < 48) {   // the geometric sums of the batch's entries
        const int e = lane / 6, k = lane - 6 * e;
        recs[e * kRecLds + k] = geo[e * kGeoStride + k];
      }
      const int er4 = lane >> 3, q4 = lane & 7;
      const float4 v4 = *(const float4*)(recs + er4 * kRecLds + 4 * q4);
      const uint32_t sl = (uint32_t)__builtin_amdgcn_ds_bpermute(er4 * 4, (int)slotv);
      // quarters 0..6 hold the kPartials values; the eighth is padding that
      // the reduction never reads, so it is not written
      static_assert(kPartials <= 28, "the partials fit in seven 16-byte quarters");
      if (er4 < nb && q4 < 7) {
        *(float4*)(partials + (size_t)sl * kSlotFloats + 4 * q4) = v4;
        if (q4 == 0) mask[sl] = 1;
      }
      // the record reads above precede the next batch's weight writes
      asm volatile("" ::: "memory");
      nb = 0;
    };
    // the list entries of the next chunk are requested a chunk ahead
    uint32_t rid_n = 0;
    if (kmax - lane >= (int)kbeg) rid_n = vals[kmax - lane];
    for (int top = kmax; top >= (int)kbeg; top -= 64) {
      // lane l takes entry top - l (the list backwards) and decides whether
      // the wave visits it
      const int kl = top - lane;
      const uint32_t rid_l = rid_n;
      bool hit = false;
      if (kl >= (int)kbeg) {
        const GeomRec g_l = load_rec_whole(geom + rid_l);
        hit = block_in_bbox(g_l.bbox, bx, by) && cull_hit(g_l, bx, by, st.cutoff2, st.log2_alpha_min);
      }
      if (kl - 64 >= (int)kbeg) rid_n = vals[kl - 64];
      uint64_t hm = __builtin_amdgcn_ballot_w64(hit);
      while (hm) {
        const uint32_t j = (uint32_t)__builtin_ctzll(hm);
        hm &= hm - 1ull;
        const int k = top - (int)j;
        const uint32_t rid = __builtin_amdgcn_readlane(rid_l, j);
        // the entry's three records are requested together, before the
        // evaluation, so their latencies overlap (the appearance and the slot
        // base are not needed when no lane contributes, but loading them
        // anyway costs less than a second round trip when one does)
        const GeomRec gr = *(const GeomRec*)((const char*)geom + (rid << 5));
        uint32_t yw[BF16 ? 10 : 20];
        load_app_words<BF16>(app, rid & npad_mask, yw);
        const uint32_t sbase = *(const uint32_t*)((const char*)slot_base + (rid << 2));
        // the compiler would sink the appearance and slot-base loads below the
        // no-contribution exit, a second round trip after the evaluation's;
        // using every loaded word here, before the geometry's first use,
        // keeps the three requests and their one wait together
        asm volatile("" ::"s"(sbase));
#pragma unroll
        for (int k = 0; k < (BF16 ? 10 : 20); ++k) asm volatile("" ::"s"(yw[k]));
        const uint64_t lm = __builtin_amdgcn_ballot_w64(k <= last);   // lanes this entry can reach
        if (CNT) {
          n_eval += (uint32_t)__popcll(lm);
          ++n_ent;
        }
        const int bx0 = (int)(gr.bbox & 255u), by0 = (int)((gr.bbox >> 16) & 255u);
        const float dx = (float)(px - 8 * bx0) - gr.mx;
        const float dy = (float)(py - 8 * by0) - gr.my;
        const Eval e = eval_entry(dx, dy, gr.qa, gr.qb2, gr.qc, gr.o, st.cutoff2, st.alpha_max, st.alpha_min);
        // (k <= last) && e.pass, as a mask of single-comparison ballots and
        // back as a lane predicate (no VALU spent on the conversion)
        const uint64_t cmask = lm & __builtin_amdgcn_ballot_w64(e.m2 <= st.cutoff2) &
                               __builtin_amdgcn_ballot_w64(e.alpha >= st.alpha_min);
        if (cmask == 0ull) continue;
        const bool con = __builtin_amdgcn_inverse_ballot_w64(cmask);
        if (CNT) {
          n_con += (uint32_t)__popcll(cmask);
          ++n_wr;
        }
        float y[20];
        y_from_words<BF16>(yw, y);
        y[3] = gr.z;
        float vv[6];
        {
          const float rinv = __builtin_amdgcn_rcpf(1.f - e.alpha);
          const float Tp = Tc * rinv;
          const float w = e.alpha * Tp;
          float gy = 0.f;
          if (kDotGy) {
            float fs = 0.f;
#pragma unroll
            for (int k = 0; k < 8; ++k)
              fs = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, yw[2 + k]),
                                                   __builtin_bit_cast(bf16x2_t, sg2[k]), fs, false);
            gy = gscale[2] * fs;
#pragma unroll
            for (int c = 0; c < 4; ++c) gy = __builtin_fmaf(g[c], y[c], gy);
          } else {
#pragma unroll
            for (int c = 0; c < 20; ++c) gy = __builtin_fmaf(g[c], y[c], gy);
          }
          const float dal = Tp * gy - (UPM == UP_EXPLICIT ? sB + gTT : sB) * rinv;   // gT = 0 otherwise
          const float wc = con ? w : 0.f;
          sB = con ? __builtin_fmaf(w, gy, sB) : sB;
          Tc = con ? Tp : Tc;
          const float dgeo = (con && !(e.araw > st.alpha_max)) ? dal : 0.f;
          // dL/dm2 per pixel is -1/2 dgeo alpha; the slot keeps the moments
          // of dgeo alpha over the pixel offsets (the factor -1/2 and the
          // conic's entries are per Gaussian, so they are applied once to
          // the summed moments in the projection backward)
          const float dm2 = dgeo * e.alpha;
          const float mxd = dm2 * dx, myd = dm2 * dy;
          vv[0] = mxd;
          vv[1] = myd;
          vv[2] = mxd * dx;
          vv[3] = mxd * dy;
          vv[4] = myd * dy;
          vv[5] = dgeo * e.G;
          // wc = hi + mid + lo exactly: each term keeps the top 8 significant
          // bits of what is left (truncation), so each is a BF16 value
          const float whi = __uint_as_float(__float_as_uint(wc) & 0xffff0000u);
          const float r1 = wc - whi;
          const float wmid = __uint_as_float(__float_as_uint(r1) & 0xffff0000u);
          const float wlo = r1 - wmid;
          wz[nb * kZRow + lane] = (unsigned short)(__float_as_uint(whi) >> 16);
          wz[(8 + nb) * kZRow + lane] = (unsigned short)(__float_as_uint(wmid) >> 16);
          wz[(16 + nb) * kZRow + lane] = (unsigned short)(__float_as_uint(wlo) >> 16);
        }
        const uint32_t bb = gr.bbox;
        const uint32_t bw = ((bb >> 8) & 255u) - (bb & 255u) + 1u;
        const uint32_t slot = sbase + (by - (uint32_t)by0) * bw + (bx - (uint32_t)bx0);
        const float s6 = transpose_reduce6(vv, lane);
        // one lane per value: 0, 8, 16, 32, 40, 48 (24 and 56 repeat 8 and 40)
        if ((lane & 7) == 0 && (lane & 24) != 24) geo[nb * kGeoStride + red6_index(lane)] = s6;
        slotv = lane == nb ? slot : slotv;   // lane nb: this entry's slot
        ++nb;
        if (nb == 8) flush();
      }
    }
    if (nb > 0) flush();
  }
  if (CNT && lane == 0) {
    atomicAdd(&cnt->bwd_evals, (unsigned long long)n_eval);
    atomicAdd(&cnt->bwd_contrib, (unsigned long long)n_con);
    atomicAdd(&cnt->bwd_entries, (unsigned long long)n_ent);
    atomicAdd(&cnt->bwd_written, (unsigned long long)n_wr);
  }
}



// Per-Gaussian sum of the backward's partials.  Visible (view, Gaussian) c
// owns the slot range [slot_off[c], slot_off[c + 1]) (the last one ends at
// n_slots); a slot holds a partial only where the backward set its mask byte.
// Each half of a wave takes one c (waves loop over pairs of c, grid-stride,
// persistent grid).  Lane l of a half sums value l of every written slot, in
// slot order, so a half reads each slot as one contiguous 128-byte access
// and needs no exchange between lanes: per window of 32 slots, lane l tests
// slot l's mask byte, a ballot gives the half its written slots, and the
// half walks them lowest first in batches (2 kSegBatch while that many are
// left, else kSegBatch), each batch's loads requested before the first is
// added.  A fixed order, so results are deterministic.
constexpr int kSegBatch = 8;
__global__ void __launch_bounds__(256) k_seg_reduce(const uint32_t* __restrict__ slot_off,
                                                    const float* __restrict__ partials,
                                                    uint8_t* __restrict__ mask,
                                                    const Counters* __restrict__ cnt,
                                                    float* __restrict__ grad2d) {
  const int lane = threadIdx.x & 63;
  if (cnt->overflow) return;
  const uint32_t nv = cnt->n_visible, ns = cnt->n_slots;
  const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
  const uint32_t w0 = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const uint32_t half = (uint32_t)lane >> 5, hl = (uint32_t)lane & 31u;
  // The slot range of the pair two ahead and the first mask byte of the
  // next pair are requested before the current pair is summed, so a pair
  // waits on one memory round trip (its records) instead of three (range,
  // mask, records).  The requests are unconditional, at clamped indices, and
  // their words are combined only when the pair comes up, so nothing waits
  // on them early.
  if (nv == 0u) return;
  const uint32_t step = 2 * n_waves;
  auto req = [&](uint32_t cc, uint32_t& b, uint32_t& e) {   // raw words of pair member cc
    const uint32_t ci = min(cc, nv - 1u);
    b = slot_off[ci];
    e = slot_off[min(ci + 1u, nv - 1u)];
  };
  auto range = [&](uint32_t cc, uint32_t braw, uint32_t eraw, uint32_t& b, uint32_t& l) {
    const bool valid = cc < nv;
    b = valid ? braw : 0u;
    l = valid ? (cc + 1u < nv ? eraw : ns) - braw : 0u;
  };
  auto req_mask = [&](uint32_t b, uint32_t l) {   // the byte of this lane's first slot (or slot 0)
    return mask[l > 0u ? b + min(hl, l - 1u) : 0u];
  };
  uint32_t rb0, re0, rb1, re1;
  req(2 * w0 + half, rb0, re0);
  req(2 * w0 + step + half, rb1, re1);
  uint32_t b0, l0;
  range(2 * w0 + half, rb0, re0, b0, l0);
  uint32_t mraw0 = req_mask(b0, l0);
  for (uint32_t c0 = 2 * w0; c0 < nv; c0 += step) {
    const uint32_t c = c0 + half;
    uint32_t rb2, re2;
    req(c0 + 2 * step + half, rb2, re2);
    uint32_t b1, l1;
    range(c0 + step + half, rb1, re1, b1, l1);
    const uint32_t mraw1 = req_mask(b1, l1);
    // the requests above stay ahead of the summing below (no memory operation
    // moves across this point)
    asm volatile("" ::: "memory");
    const uint32_t base = b0, len = l0;
    const uint32_t maxlen = __builtin_amdgcn_readfirstlane(max(len, (uint32_t)__shfl_xor((int)len, 32, 64)));
    // the slot a lane with nothing to add reads: the half's last one read
    // (already in cache), slot 0 before the first (read by every wave)
    uint32_t last = 0u;
    float acc = 0.f;
    for (uint32_t o = 0; o < maxlen; o += 32) {
      const uint32_t sl = base + o + hl;
      // the window's first byte per lane is the one requested a pair ago
      const bool written = o == 0u ? (hl < len && mraw0 != 0u) : (o + hl < len && mask[sl] != 0);
      if (written) mask[sl] = 0;   // cleared for the next backward over these slots
      const uint64_t bal = __builtin_amdgcn_ballot_w64(written);
      const uint32_t lo = (uint32_t)bal, hi = (uint32_t)(bal >> 32);
      uint32_t mine = half ? hi : lo;
      const uint32_t nmax = max((uint32_t)__builtin_popcount(lo), (uint32_t)__builtin_popcount(hi));
      const uint32_t sb = base + o;
      auto batch = [&](auto nb_tag) {
        constexpr int NB = decltype(nb_tag)::value;
        float t[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          // the lowest written slot left (once none is, the last slot read,
          // whose value is dropped)
          const bool v = mine != 0u;
          last = v ? sb + (uint32_t)__builtin_ctz(mine) : last;
          mine &= mine - 1u;
          const float x = partials[(size_t)last * kSlotFloats + hl];
          t[j] = v ? x : 0.f;
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) acc += t[j];
      };
      // long runs (a view where a Gaussian covers many blocks) in batches of
      // 2 kSegBatch, the rest in batches of kSegBatch
      uint32_t k = 0;
      for (; k + 2 * kSegBatch <= nmax; k += 2 * kSegBatch) batch(std::integral_constant<int, 2 * kSegBatch>());
      for (; k < nmax; k += kSegBatch) batch(std::integral_constant<int, kSegBatch>());
    }
    if (c < nv && hl < (uint32_t)kPartials) grad2d[(size_t)c * kPartials + hl] = acc;
    b0 = b1;
    l0 = l1;
    mraw0 = mraw1;
    rb1 = rb2;
    re1 = re2;
  }
}

}  // namespace

template <bool BF16, bool CNT, bool NC>
static void launch_fwd_t(const Settings& st, const ViewDesc* views, const ViewImages* out, const uint2* ranges,
                         const uint32_t* vals, const GeomRec* geom, const void* app, uint32_t npad_mask,
                         const uint32_t* items, const uint32_t* qoff, int64_t n_items, Counters* cnt,
                         int waves_per_group, int32_t* last_idx, float* T_state, hipStream_t s) {
  const int threads = 64 * waves_per_group;
  int dev = 0, cus = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int occ = 1;
  const size_t lds = BF16 ? (size_t)waves_per_group * kFwdWaveLds : 0;
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_raster_fwd<BF16, CNT, NC>, threads, lds);
  int64_t grid = (int64_t)cus * (occ > 0 ? occ : 1);
  const int64_t need = (n_items + waves_per_group - 1) / waves_per_group;
  if (grid > need) grid = need;
  if (grid < kQueues) grid = kQueues;   // every queue needs a workgroup (index mod kQueues) to drain it
  hipLaunchKernelGGL((k_raster_fwd<BF16, CNT, NC>), dim3((unsigned)grid), dim3(threads), lds, s, st, views, out,
                     ranges, vals, geom, app, npad_mask, items, qoff, (uint32_t)n_items, cnt, last_idx, T_state);
}

void launch_raster_fwd(const Settings& st, const ViewDesc* views, const ViewImages* out, const uint2* ranges,
                       const uint32_t* vals, const GeomRec* geom, const void* app, int app_bf16,
                       uint32_t npad_mask, const uint32_t* items, const uint32_t* qoff, int64_t n_items,
                       Counters* cnt, int waves_per_group, int32_t* last_idx, float* T_state, int n_contrib,
                       hipStream_t s) {
  if (n_items <= 0) return;
#define LGS_FWD(B, K, N)                                                                                     \
  launch_fwd_t<B, K, N>(st, views, out, ranges, vals, geom, app, npad_mask, items, qoff, n_items, cnt,       \
                        waves_per_group, last_idx, T_state, s)
#define LGS_FWD_N(B, K)        \
  if (n_contrib) LGS_FWD(B, K, true); \
  else LGS_FWD(B, K, false)
  if (app_bf16) {
    if (st.count) LGS_FWD_N(true, true);
    else LGS_FWD_N(true, false);
  } else {
    if (st.count) LGS_FWD_N(false, true);
    else LGS_FWD_N(false, false);
  }
#undef LGS_FWD_N
#undef LGS_FWD
}

template <bool BF16, int UPM, bool CNT>
static void launch_bwd_t(const Settings& st, const ViewDesc* views, const ViewImages* upstream,
                         const ViewImages* fwd_out, const ViewImages* targets, const float* loss_w,
                         const uint2* ranges, const uint32_t* vals, const GeomRec* geom, const void* app,
                         uint32_t npad_mask, const uint32_t* items, const uint32_t* qoff, int64_t n_items,
                         Counters* cnt, int waves_per_group, const int32_t* last_idx, const float* T_state,
                         const uint32_t* slot_base, float* partials, uint8_t* mask, hipStream_t s) {
  const int threads = 64 * waves_per_group;
  const size_t lds = (size_t)waves_per_group * bwd_wave_lds_bytes(UPM);
  int dev = 0, cus = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int occ = 1;
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_raster_bwd<BF16, UPM, CNT>, threads, lds);
  int64_t grid = (int64_t)cus * (occ > 0 ? occ : 1);
  const int64_t need = (n_items + waves_per_group - 1) / waves_per_group;
  if (grid > need) grid = need;
  if (grid < kQueues) grid = kQueues;   // every queue needs a workgroup (index mod kQueues) to drain it
  hipLaunchKernelGGL((k_raster_bwd<BF16, UPM, CNT>), dim3((unsigned)grid), dim3(threads), lds, s, st, views,
                     upstream, fwd_out, targets, loss_w, ranges, vals, geom, app, npad_mask, items, qoff,
                     (uint32_t)n_items, cnt, last_idx, T_state, slot_base, partials, mask);
}

void launch_raster_bwd(int up_mode, const Settings& st, const ViewDesc* views, const ViewImages* upstream,
                       const ViewImages* fwd_out, const ViewImages* targets, const float* loss_w,
                       const uint2* ranges, const uint32_t* vals, const GeomRec* geom, const void* app,
                       int app_bf16, uint32_t npad_mask, const uint32_t* items, const uint32_t* qoff,
                       int64_t n_items, Counters* cnt, int waves_per_group, const int32_t* last_idx,
                       const float* T_state, const uint32_t* slot_base, float* partials, uint8_t* mask,
                       hipStream_t s) {
  if (n_items <= 0) return;
#define LGS_BWD(B, M)                                                                                     \
  (st.count ? launch_bwd_t<B, M, true>(st, views, upstream, fwd_out, targets, loss_w, ranges, vals, geom, app,  \
                                       npad_mask, items, qoff, n_items, cnt, waves_per_group, last_idx,      \
                                       T_state, slot_base, partials, mask, s)                                 \
            : launch_bwd_t<B, M, false>(st, views, upstream, fwd_out, targets, loss_w, ranges, vals, geom,  \
                                        app, npad_mask, items, qoff, n_items, cnt, waves_per_group, last_idx, \
                                        T_state, slot_base, partials, mask, s))
  if (app_bf16) {
    if (up_mode == UP_L1) LGS_BWD(true, UP_L1);
    else if (up_mode == UP_RGB) LGS_BWD(true, UP_RGB);
    else LGS_BWD(true, UP_EXPLICIT);
  } else {
    if (up_mode == UP_L1) LGS_BWD(false, UP_L1);
    else if (up_mode == UP_RGB) LGS_BWD(false, UP_RGB);
    else LGS_BWD(false, UP_EXPLICIT);
  }
#undef LGS_BWD
}

void launch_seg_reduce(const uint32_t* slot_off, const float* partials, uint8_t* mask,
                       const Counters* cnt, int64_t n_max, float* grad2d, hipStream_t s) {
  if (n_max <= 0) return;
  int dev = 0, cus = 256, occ = 1;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_seg_reduce, 256, 0);
  int64_t grid = (int64_t)cus * (occ > 0 ? occ : 1);
  const int64_t need = (n_max + 7) / 8;   // two visible ids per wave
  if (grid > need) grid = need;
  hipLaunchKernelGGL(k_seg_reduce, dim3((unsigned)grid), dim3(256), 0, s, slot_off, partials, mask, cnt, grad2d);
}

}  // namespace lgs

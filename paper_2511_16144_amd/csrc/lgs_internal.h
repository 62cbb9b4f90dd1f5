// Internal declarations shared by the HIP translation units of the
// rasterizer: device-side records, per-view descriptors, launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace lgs {

// Pixel blocks are 8x8: one wave64 renders one block, one pixel per lane.
constexpr int kBlock = 8;
constexpr int kMaxSide = 2048;          // 8-bit block coordinates in records
constexpr int kChannels = 20;           // RGB 3 + depth 1 + feature 16
constexpr int kPartials = 26;           // geometric moments 5, opacity 1, y 20
constexpr int kSlotFloats = 32;         // a backward slot record: the kPartials floats padded to 128 bytes

// Per-view constants, shared by every stage (device array of n_views).
struct ViewDesc {
  double fx, fy, cx, cy;
  double R[9], t[3];
  double limx, limy;          // Jacobian clamp limits on x/z, y/z
  int32_t W, H;
  int32_t blocks_x, blocks_y; // 8x8 blocks
  int32_t tiles_x, tiles_y;   // binning tiles
  int32_t tile_off;           // first global tile id of this view
  int32_t item_off;           // first work item (8x8 block) of this view
  int32_t pix_off;            // first pixel of this view in packed state
  int32_t pad;
};

// Output / upstream image pointers of one view.
struct ViewImages {
  float *rgb, *depth, *feat, *T;
  int32_t *n_contrib;
};

// One view of the mapping loss (rendered and observed images, gradient
// planes, FP32 [C][H][W]) and its scale factors:
//   s_l1 = w_rgb (1 - lam) / (3HW), s_ssim = w_rgb lam / (3HW),
//   s_d = w_depth / (HW), s_f = w_feat / (D HW).
// Colour work-groups of the view: [blk_off, blk_off + n_blk), three per
// 32 x 32 tile (one per channel); depth + feature work-groups: [df_off,
// df_off + n_df), one per run of kLossDfPixels pixels; vec4: the depth and
// feature planes allow 16-byte accesses.
struct LossView {
  const float *x, *xt, *d, *dt, *f, *ft;
  float *gx, *gd, *gf;
  int32_t W, H, tiles_x, blk_off, n_blk, df_off, n_df, vec4, nf, pad;   // nf: feature planes D
  float s_l1, s_ssim, s_d, s_f;
};
constexpr int kLossDfPixels = 2048;
constexpr int kSsimRadius = 5;   // 11 x 11 SSIM window
struct LossConsts {
  float w[2 * kSsimRadius + 1];  // normalised 1-D window weights
  float c1, c2;
  int32_t ssim;                  // 0: lam = 0, the SSIM stencil is skipped
  int32_t n_views;
};

// Screen-space record of one visible (view, Gaussian), 32 bytes, read by the
// compositing kernels through scalar loads (wave-uniform).
//   mx, my : mean' relative to the pixel origin (8 bx0, 8 by0) of its bbox
//   qa, qb2, qc : conic (Q_xx, 2 Q_xy, Q_yy)
//   o      : opacity
//   z      : camera depth (the depth channel value)
//   bbox   : block rectangle bx0 | bx1 << 8 | by0 << 16 | by1 << 24 (inclusive)
struct __attribute__((aligned(32))) GeomRec {
  float mx, my, qa, qb2, qc, o, z;
  uint32_t bbox;
};

// The language features of dimension D are processed in groups of 16
// channels (the last group of D = 8 has 8): the compositing kernels carry
// RGB + depth + one group; further groups re-run them with that group's
// appearance records (blend weights do not depend on the features).
constexpr int kFeatGroup = 16;
struct Settings {
  float z_near, eps2d, fov_clamp, alpha_max, alpha_min, T_eps, cutoff2;
  int32_t tile, tile_shift;   // tile side and log2(tile / 8)
  int32_t feat_dim;           // D: feature planes of the inputs
  int32_t nfeat;              // feature channels of the group being processed (8 or 16)
  int32_t count;              // 1: the compositing kernels' profiling variants, which count their work
  float log2_alpha_min;       // log2(alpha_min), for the compositing kernels' block cull
};

// Device-resident counters of one forward (written by kernels, read by
// kernels; the host reads n_pairs in eager mode).
// Work items of the compositing kernels are split into kQueues queues, one
// per XCD (the GPU dispatches workgroup i to XCD i mod 8): all blocks of a
// binning tile go to the same queue, so the tile's list is fetched into one
// XCD's L2 and reused there by the blocks that walk it.
#ifndef LGS_XCD_QUEUES
#define LGS_XCD_QUEUES 1
#endif
constexpr int kQueues = 8;

constexpr int kLineWords = 32;   // one 128-byte line per queue counter

struct __attribute__((aligned(128))) Counters {
  uint32_t n_visible;   // M
  uint32_t n_pairs;     // P
  uint32_t n_slots;     // S
  uint32_t overflow;    // set when P exceeds the pair capacity
  uint32_t n_pairs_eff; // n_pairs, or 0 after an overflow
  uint32_t n_slots_eff; // n_slots, or 0 after an overflow
  uint32_t pad0, pad1;
  // work actually done by the compositing kernels (one atomic per wave):
  // (pixel, entry) evaluations and contributions, the list entries a wave
  // visited (its records were loaded), forward and backward, and the
  // backward's partial records written
  unsigned long long fwd_evals, fwd_contrib, fwd_entries;
  unsigned long long bwd_evals, bwd_contrib, bwd_entries, bwd_written;
  uint32_t pad2[42];   // the queue counters below start on a 128-byte line
  // persistent-kernel work counters, queue q at word q * kLineWords, each on
  // its own line so that the queues' atomics do not serialise on one address
  uint32_t work_q[kQueues * kLineWords];    // forward
  uint32_t work_qb[kQueues * kLineWords];   // backward
};
static_assert(offsetof(Counters, work_q) % 128 == 0, "queue counters must start on a 128-byte line");

// Queue of the items of binning tile t (global tile index) in the raster
// and list-length orders (settings.order 0 and 1): neighbouring tiles go to
// different XCDs.
__host__ __device__ inline uint32_t tile_queue(uint32_t t) { return LGS_XCD_QUEUES ? (t % kQueues) : 0u; }
// Spatial order (settings.order 2): the views are cut into super-tiles of
// kSuperPx x kSuperPx pixels and each super-tile goes to one queue (a
// lattice over (super-tile x, y, view), so that neighbouring super-tiles go
// to different XCDs); inside a queue items run in descending tile-list
// length as in order 1.  The tiles of one region then share their XCD's L2
// for the records of the Gaussians they have in common.
constexpr int kSuperPx = 128;
__host__ __device__ inline uint32_t super_queue(uint32_t v, uint32_t bx, uint32_t by) {
  constexpr uint32_t sh = 4;   // log2(kSuperPx / 8): 8x8 blocks per super-tile side
  static_assert((8u << sh) == (uint32_t)kSuperPx, "super-tile side");
  return LGS_XCD_QUEUES ? (((bx >> sh) + 3u * (by >> sh) + 5u * v) % (uint32_t)kQueues) : 0u;
}

// ---------------------------------------------------------------------------
// launchers (each defined next to its kernels)
// ---------------------------------------------------------------------------
// projection (K1)
void launch_project(const Settings& st, const ViewDesc* views, int n_views,
                    const float* means, const float* log_scales, const float* quats,
                    const float* logits, const void* rgb, const void* feat, int app_bf16,
                    int64_t n, uint32_t npad_shift,
                    GeomRec* geom, uint32_t* cnt_t, uint32_t* cnt_b, uint32_t* dkey,
                    void* app, Counters* cnt, hipStream_t s);   // also zeroes *cnt (the step's first kernel)

// scans
size_t scan_temp_bytes(int64_t n);
enum ScanInput { SCAN_FLAG_NONZERO = 0, SCAN_VALUE = 1, SCAN_GATHER = 2 };
// out[i] = exclusive prefix of in(i); total written to *total.
// in(i) = (src[i] != 0) / src[i] / src[idx[i]] by mode; n read from *n_dev
// when n_dev != nullptr (n_max bounds the grid), else n_max.
// out_at_idx (gather scans only, or NULL): each value also written at its
// source index, out_at_idx[idx[i]] = out[i].  A gather scan also uses out
// to hold the gathered values between its two passes, so out must not
// overlap src or idx.
// Compaction (flag scans only, ent == nullptr for none; not together with
// out_at_idx): for every flagged item i, with c = out[i]: ent[c] =
// ent_copy[c] = i and keys[c] = key_src[i].
struct Compact {
  const uint32_t* key_src = nullptr;
  uint32_t* ent = nullptr;
  uint32_t* ent_copy = nullptr;
  uint32_t* keys = nullptr;
};
void launch_scan(int mode, const uint32_t* src, const uint32_t* idx, uint32_t* out,
                 uint32_t* total, const uint32_t* n_dev, int64_t n_max,
                 void* temp, hipStream_t s, uint32_t* out_at_idx = nullptr, Compact cp = Compact());

// pair emission (load-balanced over pairs), tile ranges
void launch_emit(const GeomRec* geom, const ViewDesc* views, const uint32_t* srid,
                 const uint32_t* off_t, const Counters* cnt, int64_t pair_grid_max,
                 int64_t cap_pairs, int npad_shift, int tile_shift,
                 uint32_t* keys, uint32_t* vals, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_zero2_u32(uint32_t* p, int64_t np, uint32_t* q, int64_t nq, hipStream_t s);
void launch_fill_u8(uint8_t* p, uint8_t v, const uint32_t* n_dev, int64_t n_max, hipStream_t s);
void launch_tile_ranges(const uint32_t* keys, const Counters* cnt, int64_t grid_max,
                        uint2* ranges, hipStream_t s);
// the step's overflow flag and effective counts; also zeroes zero[0 .. n_zero)
void launch_set_overflow(Counters* cnt, uint64_t cap_pairs, uint64_t cap_slots, uint32_t* zero, int64_t n_zero,
                         hipStream_t s);
// radix sort (LSD, 8-bit digits, stable)
size_t radix_temp_bytes(int64_t n_max);
void radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                    const uint32_t* n_dev, int64_t n_max, int begin_bit, int end_bit,
                    void* temp, hipStream_t s, bool* result_in_alt);
void radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                    const uint32_t* n_dev, int64_t n_max, int begin_bit, int end_bit,
                    void* temp, hipStream_t s, bool* result_in_alt);

// work queue ordering (blocks by descending tile-list length): each queue's
// tiles re-sorted by the length of their list (counting sort on coarse
// length buckets, one work-group per queue), a tile's blocks kept together;
// qoff: the queues' item offsets, tiles: the queue-major tile table, tq: its
// queues' tile offsets (kQueues + 1); returns out
struct TileItems {
  uint32_t first;   // index of the tile's first item in the static table
  uint32_t count;   // its blocks (items)
  uint32_t tile;    // global tile id
  uint32_t queue;
};
uint32_t* launch_order_items(const uint2* ranges, const uint32_t* items, const uint32_t* qoff, const TileItems* tiles,
                             const uint32_t* tq, int64_t n_tiles, uint32_t* out, hipStream_t s);

// compositing
void launch_raster_fwd(const Settings& st, const ViewDesc* views, const ViewImages* out,
                       const uint2* ranges, const uint32_t* vals, const GeomRec* geom,
                       const void* app, int app_bf16, uint32_t npad_mask,
                       const uint32_t* items, const uint32_t* qoff, int64_t n_items, Counters* cnt,
                       int waves_per_group, int32_t* last_idx, float* T_state, int n_contrib,
                       hipStream_t s);   // n_contrib: some view's out table asks for contributor counts
// Upstream of the backward compositing kernel: dL/dY given per channel
// (upstream), the L1 loss gradient formed from the forward's images and the
// targets (loss_w), or the colour channels given and depth + features from
// the L1 residual (the D-SSIM loss, whose colour gradient a kernel writes).
enum UpMode { UP_EXPLICIT = 0, UP_L1 = 1, UP_RGB = 2 };
// LDS upstream rows per wave: hi rows for the 20 channels plus lo rows for
// the channels given as FP32 values
__host__ __device__ constexpr int bwd_upstream_rows(int up_mode) {
  return up_mode == UP_L1 ? 20 : (up_mode == UP_RGB ? 23 : 40);
}
void launch_raster_bwd(int up_mode, const Settings& st, const ViewDesc* views, const ViewImages* upstream,
                       const ViewImages* fwd_out, const ViewImages* targets, const float* loss_w,
                       const uint2* ranges, const uint32_t* vals, const GeomRec* geom,
                       const void* app, int app_bf16, uint32_t npad_mask,
                       const uint32_t* items, const uint32_t* qoff, int64_t n_items, Counters* cnt,
                       int waves_per_group, const int32_t* last_idx, const float* T_state,
                       const uint32_t* slot_base, float* partials, uint8_t* mask, hipStream_t s);

// mapping loss (L1 + D-SSIM) and its gradient: the colour channels (L1 and
// SSIM stencil), the depth and feature channels (L1), and the per-view terms
// {mean|I-I*|, 1 - SSIM (0 when ssim = 0), mean|D-D*|, mean|F-F*|} from the
// work-groups' partial sums
int64_t loss_blocks(int W, int H);
int64_t loss_df_blocks(int W, int H);
int loss_tiles_x(int W);
void launch_loss_rgb(const LossView* views, const LossConsts& k, int64_t n_blocks, float2* partials,
                     hipStream_t s);
void launch_loss_df(const LossView* views, int n_views, int64_t n_blocks, float2* partials, hipStream_t s);
void launch_loss_terms(const LossView* views, int n_views, int ssim, const float2* part_rgb,
                       const float2* part_df, float* terms, hipStream_t s);

// feature decoder (1x1 convolution 16 -> C) and its L1 distillation loss
// over one or more views (each view's loss normalised by its own C H W, the
// views' losses summed): dL/dF per view, dL/dW, dL/db and the loss.  Every
// work-group works on one view's chunks; part holds grid x part_stride
// floats of per-work-group partial sums (dW [C][16], db [C], loss), already
// times the view's scale
constexpr int kDecMaxViews = 16;
struct DecView {
  const float* feat;                   // F [16][n]
  const void* target;                  // F* [C][n], BF16 or FP32
  float* grad_feat;                    // dL/dF [16][n]
  int64_t n;                           // pixels
  float scale;                         // w_feat / (C n)
  int32_t vec;                         // targets allow 8-element vector loads (n % 8 == 0, 16-B base)
  int32_t g0, groups;                  // its work-groups g0 .. g0 + groups - 1 (decoder_assign)
};
struct DecArgs {
  const float *weight, *bias;          // W [C][16], b [C]
  float *grad_weight, *grad_bias, *loss;
  int64_t part_stride;                 // >= 17 C + 1
  int32_t C;                           // 256 or 512
  int32_t n_views;                     // 1 .. kDecMaxViews
  DecView v[kDecMaxViews];
};
bool decoder_dim_ok(int C);
// shares out the work-groups of the launch among the views (at most one per
// CU and at most `cap` in all, unless there are more views; at least one per
// view, at most one per 32-pixel chunk) and returns the grid
int decoder_assign(DecArgs& a, int cap);
void launch_decoder(const DecArgs& a, int target_bf16, float* part, int grid, hipStream_t s);

// language-guided pruning (K nearest neighbours in a uniform grid of cell
// side tau_dist) and the geometric criteria
struct PruneArgs {
  const float *means, *logits, *log_scales;   // [3][n], [n], [3][n]
  const void* feat;                           // [16][n], FP32 or BF16
  int32_t feat_bf16, k;                       // k <= prune_k_max()
  int64_t n, n_valid;                         // Gaussians; those with a grid cell (sorted first)
  double tau2, inv_cell, tau_sim;             // tau_dist^2, 1 / tau_dist, tau_sim
  double logit_min, log_scale_max;            // log(o / (1 - o)) of min_opacity, log(max_scale)
};
int prune_k_max();
size_t prune_temp_bytes(int64_t n);
void launch_prune_keys(const PruneArgs& a, uint64_t* keys, uint32_t* vals, uint8_t* geo, uint32_t* range_err,
                       hipStream_t s);
void launch_prune_count_valid(const uint64_t* keys, int64_t n, int64_t* n_valid, hipStream_t s);
void launch_prune_knn(const PruneArgs& a, const uint64_t* keys, const uint32_t* vals, uint8_t* sem, hipStream_t s);
void launch_prune_final(int64_t n, const uint8_t* sem, const uint8_t* geo, uint8_t* mask,
                        unsigned long long* counts, hipStream_t s);

// feature groups beyond the first: appearance records (RGB 0, the group's
// features), the geometric partials of a group's backward added to the
// first group's, and a group's feature gradients summed over views
void launch_pack_app_group(const void* feat_g, int nfeat, int app_bf16, int64_t n, void* app, hipStream_t s);
void launch_group_geo_acc(const float* grad2d_g, const Counters* cnt, int64_t n_max, float* geo_acc, int first,
                          hipStream_t s);
void launch_group_geo_add(float* grad2d, const Counters* cnt, int64_t n_max, const float* geo_acc, hipStream_t s);
void launch_group_feat_grad(int n_views, int64_t n, uint32_t npad_shift, const Counters* cnt, const uint32_t* cnt_t,
                            const uint32_t* cidx, const float* grad2d_g, int nfeat, float* g_feat_g, hipStream_t s);

// gradient reduction and projection backward
void launch_seg_reduce(const uint32_t* slot_off, const float* partials, uint8_t* mask,
                       const Counters* cnt, int64_t n_max, float* grad2d, hipStream_t s);
// workspace of launch_project_bwd for at most n_rid visible (view, Gaussian)
size_t project_bwd_temp_bytes(int64_t n_rid, int n_views);
// the projection backward: per visible (view, Gaussian) c the view's chain
// rule (ent: c's record id, in (view, Gaussian) order), then per Gaussian
// the views summed in order and the activation's chain rule
void launch_project_bwd(const Settings& st, const ViewDesc* views, int n_views, const float* means,
                        const float* log_scales, const float* quats, const float* logits, int64_t n,
                        uint32_t npad_shift, int64_t n_rid, const Counters* cnt, const uint32_t* cnt_t,
                        const uint32_t* cidx, const uint32_t* ent, const float* grad2d, float* g_means,
                        float* g_ls, float* g_q, float* g_logit, float* g_rgb, float* g_feat, float* twist,
                        void* temp, hipStream_t s);

}  // namespace lgs

// Host-side unit test of the library's planning code, for the host
// sanitizer build (AddressSanitizer + UndefinedBehaviorSanitizer on the host
// code only): this translation unit includes the runtime source, so that the
// file-local planning functions are reachable, and exports one entry point
// that the CPU test calls through ctypes.  No HIP runtime call is made.
//
// Checked: the view plan (tile, item and pixel offsets), the work-item
// tables of every order and tile size (each 8x8 block exactly once, queue
// offsets, per-tile records consistent with the items and the queue rule),
// and the autotuner cache file (round trip, replacement of a key, keys too
// long for the line buffer), and the size limits of the record addressing.
#include "../../paper_2511_16144_amd/csrc/runtime.hip"

#include <set>
#include <tuple>

namespace {

int g_fail = 0;
#define CHECK(cond)                                                                  \
  do {                                                                               \
    if (!(cond)) {                                                                   \
      fprintf(stderr, "runtime_host_test: %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++g_fail;                                                                      \
    }                                                                                \
  } while (0)

lgs_camera cam(int w, int h) {
  lgs_camera c;
  memset(&c, 0, sizeof c);
  c.width = w;
  c.height = h;
  c.fx = c.fy = 500.f;
  c.cx = 0.5f * (w - 1);
  c.cy = 0.5f * (h - 1);
  c.R_cw[0] = c.R_cw[4] = c.R_cw[8] = 1.f;
  return c;
}

void check_items(const std::vector<lgs_camera>& cams, int tile, bool spatial) {
  lgs_settings st = lgs_default_settings();
  st.tile = tile;
  const Plan P = make_plan(&st, (int32_t)cams.size(), cams.data());
  int64_t tiles = 0, items_n = 0, pix = 0;
  for (size_t v = 0; v < cams.size(); ++v) {
    const ViewDesc& d = P.views[v];
    CHECK(d.tile_off == tiles && d.item_off == items_n && d.pix_off == pix);
    CHECK(d.blocks_x == (cams[v].width + 7) / 8 && d.tiles_x == (cams[v].width + tile - 1) / tile);
    tiles += (int64_t)d.tiles_x * d.tiles_y;
    items_n += (int64_t)d.blocks_x * d.blocks_y;
    pix += (int64_t)cams[v].width * cams[v].height;
  }
  CHECK(P.n_tiles == tiles && P.n_items == items_n && P.n_pix == pix);
  const std::vector<uint32_t> it = make_items(P, tile, spatial);
  CHECK((int64_t)it.size() == P.n_items + kQueues + 1 + 4 * P.n_tiles + kQueues + 1);
  if ((int64_t)it.size() != P.n_items + kQueues + 1 + 4 * P.n_tiles + kQueues + 1) return;
  const uint32_t* qoff = it.data() + P.n_items;
  CHECK(qoff[0] == 0u && qoff[kQueues] == (uint32_t)P.n_items);
  for (int q = 0; q < kQueues; ++q) CHECK(qoff[q] <= qoff[q + 1]);
  std::set<std::tuple<uint32_t, uint32_t, uint32_t>> seen;
  const int bpt = tile / kBlock;
  for (int64_t i = 0; i < P.n_items; ++i) {
    const uint32_t x = it[i], bx = x & 255u, by = (x >> 8) & 255u, v = x >> 16;
    CHECK(v < cams.size());
    if (v >= cams.size()) continue;
    CHECK((int)bx < P.views[v].blocks_x && (int)by < P.views[v].blocks_y);
    CHECK(seen.insert(std::make_tuple(v, bx, by)).second);
  }
  CHECK((int64_t)seen.size() == P.n_items);
  const TileItems* T = (const TileItems*)(qoff + kQueues + 1);
  int64_t covered = 0;
  std::set<uint32_t> tile_ids;
  for (int64_t k = 0; k < P.n_tiles; ++k) {
    const TileItems& r = T[k];
    CHECK(r.count >= 1 && (int)r.count <= bpt * bpt && r.queue < (uint32_t)kQueues);
    CHECK(r.first >= qoff[r.queue] && r.first + r.count <= qoff[r.queue + 1]);
    CHECK(tile_ids.insert(r.tile).second);
    if (r.first + r.count > (uint32_t)P.n_items || r.queue >= (uint32_t)kQueues) continue;
    for (uint32_t j = 0; j < r.count; ++j) {
      const uint32_t x = it[r.first + j], bx = x & 255u, by = (x >> 8) & 255u, v = x >> 16;
      const ViewDesc& d = P.views[v];
      const uint32_t t = (uint32_t)d.tile_off + (by / bpt) * (uint32_t)d.tiles_x + bx / bpt;
      CHECK(t == r.tile);
      CHECK(r.queue == (spatial ? super_queue(v, bx, by) : tile_queue(t)));
    }
    covered += r.count;
  }
  CHECK(covered == P.n_items && (int64_t)tile_ids.size() == P.n_tiles);
  // the queues' tile offsets bracket exactly the records of each queue
  const uint32_t* tq = (const uint32_t*)(T + P.n_tiles);
  CHECK(tq[0] == 0u && tq[kQueues] == (uint32_t)P.n_tiles);
  for (int q = 0; q < kQueues; ++q) {
    CHECK(tq[q] <= tq[q + 1]);
    for (uint32_t k = tq[q]; k < tq[q + 1] && k < (uint32_t)P.n_tiles; ++k) CHECK(T[k].queue == (uint32_t)q);
  }
}

void check_tune_cache(const char* path) {
  remove(path);
  lgs_settings s = lgs_default_settings(), r = lgs_default_settings();
  CHECK(!tune_cache_read(path, "absent", &r));
  s.tile = 32; s.chunk = 4; s.order = 2;
  tune_cache_write(path, "n500000_bf16_d16_l1_v2_640x480_320x240", s);
  s.tile = 8; s.chunk = 1; s.order = 0;
  tune_cache_write(path, "n2000_f32_d16_l1_v1_128x96", s);
  CHECK(tune_cache_read(path, "n500000_bf16_d16_l1_v2_640x480_320x240", &r));
  CHECK(r.tile == 32 && r.chunk == 4 && r.order == 2);
  s.tile = 16; s.chunk = 2; s.order = 1;   // replacing a key keeps the others
  tune_cache_write(path, "n500000_bf16_d16_l1_v2_640x480_320x240", s);
  CHECK(tune_cache_read(path, "n500000_bf16_d16_l1_v2_640x480_320x240", &r));
  CHECK(r.tile == 16 && r.chunk == 2 && r.order == 1);
  CHECK(tune_cache_read(path, "n2000_f32_d16_l1_v1_128x96", &r));
  CHECK(r.tile == 8 && r.chunk == 1 && r.order == 0);
  // a key longer than the file's line buffer (1024 views of distinct sizes):
  // never found, and writing it must stay within the buffers
  std::vector<lgs_camera> cams;
  for (int v = 0; v < 1024; ++v) cams.push_back(cam(100 + v, 50 + v));
  lgs_gaussians g;
  memset(&g, 0, sizeof g);
  g.n = 7;
  const std::string key = tune_key(&g, (int32_t)cams.size(), cams.data());
  CHECK(key.size() > 1024);
  tune_cache_write(path, key, s);
  CHECK(!tune_cache_read(path, key, &r));
  CHECK(tune_cache_read(path, "n2000_f32_d16_l1_v1_128x96", &r));
  remove(path);
}

}  // namespace

// The size limits of w_init: the compositing kernels address the records by
// 32-bit byte offsets (32-byte geometry per (view, Gaussian), 40 / 80-byte
// appearance per Gaussian); w_init makes no HIP call before these checks.
void check_record_limits() {
  lgs_context ctx;
  const lgs_settings st = lgs_default_settings();
  const std::vector<lgs_camera> cams(4, cam(64, 48));
  auto init = [&](int64_t n, lgs_dtype dt, int views) {
    lgs_gaussians g;
    memset(&g, 0, sizeof g);
    g.n = n;
    g.appearance_dtype = dt;
    g.feat_dim = 16;
    Work W;
    return w_init(&W, &ctx, &st, &g, views, cams.data(), nullptr);
  };
  const int64_t e25 = (int64_t)1 << 25, e26 = (int64_t)1 << 26;
  CHECK(init(e25, LGS_F32, 1) == LGS_OK);                      // 80 B x 2^25 < 2^32
  CHECK(init(e25 + 1, LGS_F32, 1) == LGS_ERR_UNSUPPORTED);     // 80 B x 2^26
  CHECK(init(e26, LGS_BF16, 2) == LGS_OK);                     // 40 B x 2^26; 2 x 2^26 = 2^27 records
  CHECK(init(e26 + 1, LGS_BF16, 1) == LGS_ERR_UNSUPPORTED);    // 40 B x 2^27
  CHECK(init(e26, LGS_BF16, 3) == LGS_ERR_UNSUPPORTED);        // 3 x 2^26 records > 2^27
  CHECK(init(e25, LGS_F32, 4) == LGS_OK);                      // 4 x 2^25 = 2^27 records
}

extern "C" int lgs_host_selftest(const char* tmp_path) {
  g_fail = 0;
  const std::vector<std::vector<lgs_camera>> sets = {
      {cam(128, 96)},
      {cam(1, 1)},
      {cam(13, 7), cam(33, 17), cam(2048, 8)},
      {cam(640, 480), cam(320, 240), cam(640, 480), cam(320, 240), cam(640, 480), cam(320, 240), cam(640, 480),
       cam(320, 240)},
      {cam(1296, 968)},
      {cam(1200, 680), cam(129, 257)}};
  for (const auto& cs : sets)
    for (int tile : {8, 16, 32})
      for (bool spatial : {false, true}) check_items(cs, tile, spatial);
  check_tune_cache(tmp_path);
  check_record_limits();
  return g_fail;
}

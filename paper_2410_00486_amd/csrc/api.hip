// C ABI of the rasterizer library: plan and workspace layout, argument
// checks, the entry points of one mapping iteration, the stand-alone sort,
// and whole-iteration HIP graphs.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tilesort.h"

namespace gs {
hipError_t launch_preprocess(const Plan& P, const gs_gaussians& g, const float* cams, void* ws,
                             hipStream_t s);
hipError_t launch_bin_sort(const Plan& P, void* ws, hipStream_t s, bool defer_short_sorts = false,
                           const StepAdvance* step = nullptr, const Marks* marks = nullptr);
TileSortArgs tile_sort_args(const Plan& P, void* ws);
int64_t scan_rounds(const Plan& P);
int64_t rb_blocks(int64_t count);
int64_t rb_gen_blocks(int64_t records);
int rb_max_radix();
hipError_t launch_radix_sort(uint64_t* keys0, uint64_t* keys1, uint32_t* vals0, uint32_t* vals1,
                             const int32_t* cnt, uint32_t* hist, uint32_t* digit_tot,
                             int64_t nb_cap, int key_bits, bool iota, int* which, hipStream_t s);
hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t s);
hipError_t launch_clear_counters(const Plan& P, void* ws, hipStream_t s);
uint32_t* sorted_vals(const Plan& P, void* ws);
hipError_t launch_render_fwd(const Plan& P, void* ws, const float* cams, float* color,
                             float* depth, float* T_final, uint32_t* last,
                             const float* target_rgb, const float* target_depth,
                             float* loss_per_view, const uint32_t* order, int32_t* queue,
                             int grid, hipStream_t s, const TileSortArgs& sort = TileSortArgs{});
hipError_t launch_render_bwd(const Plan& P, void* ws, const float* cams, const float* color,
                             const float* depth, const float* T_final, const uint32_t* last,
                             const float* dL_dcolor, const float* dL_ddepth,
                             const float* target_rgb, const float* target_depth, int fused,
                             const uint32_t* sorted_vals, const uint32_t* order, int32_t* queue,
                             int grid, hipStream_t s);
hipError_t launch_project_bwd(const Plan& P, const gs_gaussians& g, const float* cams, void* ws,
                              const gs_gaussian_grads& out, float* dL_dpose, int accumulate,
                              bool zeroed, hipStream_t s);
hipError_t launch_adam(const gs_param_group* groups, int n_groups, int step, double beta1,
                       double beta2, double eps, double lambda_o, int64_t reg_count,
                       int32_t* step_dev, hipStream_t s, const uint32_t* const* vis = nullptr,
                       const int32_t* per = nullptr, const int32_t* overflow = nullptr,
                       const AdamFold* fold = nullptr);
int render_blocks_per_cu(const Plan& P, bool bwd);
int splat_blocks_per_cu(const Plan& P);
int64_t ssim_tiles(const Plan& P);
size_t densify_tmp_bytes(int64_t n);
hipError_t launch_grad_stats(const Plan& P, void* ws, float* accum, float* denom, hipStream_t s);
hipError_t launch_densify(const gs_gaussians& g, const gs_gaussian_grads& m,
                          const gs_gaussian_grads& v, const float* accum, const float* denom,
                          const float* normals, float tau_p, float eps_alpha, float percent_dense,
                          float extent, const gs_gaussian_grads& out, const gs_gaussian_grads& out_m,
                          const gs_gaussian_grads& out_v, int64_t cap, int32_t* n_out, void* tmp,
                          hipStream_t s);
hipError_t launch_gather_views(const Plan& P, const gs_view_gather& g, float* cams_out,
                               float* rgb_out, float* depth_out, hipStream_t s);
size_t spatial_order_tmp_bytes(int64_t n);
hipError_t launch_spatial_order(const float* means, int64_t n, int32_t* perm, void* tmp,
                                hipStream_t s);
hipError_t launch_gather_rows(const float* src, const int32_t* perm, int64_t n, int width,
                              float* dst, hipStream_t s);
hipError_t launch_pose_retract(const float* cams_in, const float* xi, float* cams_out,
                               int n_views, hipStream_t s);
hipError_t launch_pose_vjp(const float* xi, const float* g_delta, float* g_xi, int n_views,
                           hipStream_t s);
hipError_t launch_render_loss(const Plan& P, void* ws, const float* color, const float* depth,
                              const float* target_rgb, const float* target_depth,
                              double lambda_ssim, float* dL_dcolor, float* dL_ddepth,
                              float* loss_per_view, hipStream_t s);
}  // namespace gs

using namespace gs;

namespace {

thread_local std::string g_err;

gs_status fail(gs_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
gs_status fail(gs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

gs_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return GS_OK;
  return fail(GS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int ceil_log2(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

gs_status check_plan(const gs_plan* plan) {
  if (!plan) return fail(GS_ERR_INVALID_ARG, "plan is null");
  if (plan_of(plan)->magic != kPlanMagic) return fail(GS_ERR_INVALID_ARG, "plan is not initialised");
  return GS_OK;
}

gs_status check_ws(const Plan& P, void* ws) {
  if (!ws) return fail(GS_ERR_INVALID_ARG, "workspace is null");
  if (!aligned(ws, 256)) return fail(GS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  (void)P;
  return GS_OK;
}

gs_status check_gaussians(const Plan& P, const gs_gaussians* g) {
  if (!g) return fail(GS_ERR_INVALID_ARG, "gaussians is null");
  if (g->n != P.n) return fail(GS_ERR_INVALID_ARG, "gaussians.n (%lld) != plan n (%lld)", (long long)g->n, (long long)P.n);
  if (g->sh_degree != P.deg) return fail(GS_ERR_INVALID_ARG, "sh_degree %d != plan degree %d", g->sh_degree, P.deg);
  if (P.n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
    return fail(GS_ERR_INVALID_ARG, "a Gaussian parameter pointer is null");
  if (!aligned(g->quats, 16)) return fail(GS_ERR_INVALID_ARG, "quats must be 16-byte aligned");
  return GS_OK;
}

int device_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  });
  return cus;
}

}  // namespace

extern "C" {

int32_t gs_version(void) { return 1; }

const char* gs_status_string(gs_status s) {
  switch (s) {
    case GS_OK: return "GS_OK";
    case GS_ERR_INVALID_ARG: return "GS_ERR_INVALID_ARG";
    case GS_ERR_UNSUPPORTED: return "GS_ERR_UNSUPPORTED";
    case GS_ERR_HIP: return "GS_ERR_HIP";
    default: return "GS_ERR_UNKNOWN";
  }
}

const char* gs_last_error(void) { return g_err.c_str(); }

gs_status gs_plan_init(gs_plan* plan, int64_t n, int32_t sh_degree, int32_t n_views,
                       const int32_t* view_wh, const gs_raster_cfg* cfg, int64_t pair_capacity) {
  if (!plan || !view_wh || !cfg) return fail(GS_ERR_INVALID_ARG, "plan, view_wh and cfg must be non-null");
  std::memset(plan, 0, sizeof(*plan));
  if (n < 0) return fail(GS_ERR_INVALID_ARG, "n must be >= 0");
  if (sh_degree < 0 || sh_degree > 3) return fail(GS_ERR_UNSUPPORTED, "sh_degree must be 0..3");
  if (n_views < 1 || n_views > GS_MAX_VIEWS) return fail(GS_ERR_INVALID_ARG, "n_views must be 1..%d", GS_MAX_VIEWS);
  const int tw = cfg->tile_w, th = cfg->tile_h;
  if (!((tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 8)))
    return fail(GS_ERR_UNSUPPORTED, "tile shape %dx%d not supported (16x16, 16x8, 8x8)", tw, th);
  if (cfg->lds_batch < 32 || cfg->lds_batch > 256 || (cfg->lds_batch % 32) != 0)
    return fail(GS_ERR_UNSUPPORTED, "lds_batch must be a multiple of 32 in 32..256");
  if (cfg->chunk < 1 || cfg->chunk > 16) return fail(GS_ERR_INVALID_ARG, "chunk must be 1..16");
  if (pair_capacity < 1 || pair_capacity > INT32_MAX) return fail(GS_ERR_INVALID_ARG, "pair_capacity must be 1..2^31-1");
  Plan* P = plan_of(plan);
  P->n = n;
  P->deg = sh_degree;
  P->K = (sh_degree + 1) * (sh_degree + 1);
  P->n_views = n_views;
  P->n_rec = n * n_views;
  if (P->n_rec > INT32_MAX) return fail(GS_ERR_INVALID_ARG, "n * n_views must be < 2^31");
  P->pair_cap = pair_capacity;
  P->cfg = *cfg;
  ViewTable& vt = P->vt;
  vt.n_views = n_views;
  vt.tw = tw;
  vt.th = th;
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = view_wh[2 * v], H = view_wh[2 * v + 1];
    if (W < 1 || H < 1 || W > 16384 || H > 16384) return fail(GS_ERR_INVALID_ARG, "view %d size %dx%d out of range", v, W, H);
    ViewInfo& vi = vt.v[v];
    vi.W = W;
    vi.H = H;
    vi.tiles_x = (W + tw - 1) / tw;
    vi.tiles_y = (H + th - 1) / th;
    vi.tile_off = (int32_t)tiles;
    vi.pix_off = (int32_t)pix;
    tiles += (int64_t)vi.tiles_x * vi.tiles_y;
    pix += (int64_t)W * H;
    if (tiles > INT32_MAX / 2 || pix > INT32_MAX / 3) return fail(GS_ERR_INVALID_ARG, "too many pixels or tiles");
  }
  vt.total_tiles = (int32_t)tiles;
  vt.total_pix = pix;
  P->tile_bits = std::max(1, ceil_log2(tiles));
  P->chunks_per_view = (n + kWave - 1) / kWave;
  P->n_chunks = (int64_t)n_views * P->chunks_per_view;
  P->proj_blocks = (n + kProjThreads - 1) / kProjThreads;

  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1), 256);
    return at;
  };
  const size_t cap = (size_t)pair_capacity, nrec = (size_t)P->n_rec, T = (size_t)tiles;
  P->off_flags = take(F_COUNT * 4 * 4);
  P->off_rec = take(nrec * sizeof(Rec));
  P->off_rect = take(nrec * 8);
  P->off_tt = take(nrec * 4);
  P->off_poff = take(nrec * 4);
  P->off_chunk_cnt = take((size_t)P->n_chunks * 8);
  P->off_chunk_pre = take((size_t)P->n_chunks * 8);
  P->off_vis_list = take(nrec * 4);
  P->off_vis_clamp = take(nrec * 4);
  P->off_tile_cnt = take(T * 4);
  P->off_tile_start = take(T * 4);
  P->off_long = take(T * 16);  // (tile, list start, pairs, -) per long list
  // the per-tile binning's scattered keys, pair records and record copies
  // in list order; the radix binning has buffers of its own (below) and
  // its lists name their records
  const bool radix = (cfg->flags & GS_RADIX_BIN) != 0;
  const size_t tcap = radix ? 0 : cap;
  P->off_keys = take(cap * 8);
  P->off_scatter = take(tcap * 8);
  P->off_vals = take(cap * 4);
  P->off_pair_rec = take(tcap * 4);
  P->off_sorted_rec = take(cap * 4);
  P->off_srec = take(tcap * sizeof(Rec));
  P->off_ranges = take(T * 2 * 4);
  P->off_tile_last = take(T * 4);
  P->off_tile_loss = take(T * 2 * 4);
  P->off_grad_pair = take(cap * kPairGrad * 4);
  P->off_pose_part = take((size_t)n_views * std::max<int64_t>(P->proj_blocks, 1) * 6 * 8);
  P->off_order = take(T * 4);
  P->off_rec_terms = take(n_views > 1 ? nrec * 14 * 8 : 0);
  P->off_gp_tmp = take(n_views > 1 ? (size_t)n * 4 * 8 : 0);
  P->off_ssim_maps = take((size_t)pix * 9 * 4);
  P->off_ssim_part = take((size_t)ssim_tiles(*P) * 12 * 4);
  // splat-wise backward: bucket k of tile t uses checkpoint slot boff[t] + k,
  // boff the exclusive scan of ceil(pairs of tile / 64); at most
  // pair_capacity / 64 + tiles slots
  const bool splat = (cfg->flags & GS_SPLAT_BWD) != 0;
  P->ckpt_slots = splat ? pair_capacity / kBucket + tiles : 0;
  P->off_boff = take(splat ? (T + 1) * 4 : 0);
  P->off_bq = take((size_t)P->ckpt_slots * 2 * 8);  // two bucket queues of (tile, k)
  P->off_full_start = take(splat ? T * 4 : 0);
  P->off_half_start = take(splat ? T * 4 : 0);
  P->off_ckpt = take((size_t)P->ckpt_slots * tw * th * kStateFloats * 4);
  P->scan_rounds = scan_rounds(*P);
  P->off_scan_part = take((size_t)P->scan_rounds * 64);
  // radix binning buffers, only when the plan asks for that binning
  P->rb_rec_blocks = radix ? rb_blocks(P->n_rec) : 0;
  P->rb_pair_blocks = radix ? rb_blocks(pair_capacity) : 0;
  const size_t rrec = radix ? nrec * 4 : 0, rpair = radix ? cap * 4 : 0;
  for (int k = 0; k < 2; ++k) {
    P->off_rb_dkey[k] = take(rrec);
    P->off_rb_rid[k] = take(rrec);
    P->off_rb_tkey[k] = take(rpair);
    P->off_rb_gidx[k] = take(rpair);
    P->off_rb_ridx[k] = take(rpair);
  }
  P->off_rb_hist = take(radix ? (size_t)rb_max_radix() * 4 *
                                    std::max(P->rb_rec_blocks, P->rb_pair_blocks) : 0);
  P->off_rb_dtot = take(radix ? (size_t)rb_max_radix() * 4 : 0);
  P->off_rb_part = take(radix ? (size_t)rb_gen_blocks(P->n_rec) * 4 : 0);
  P->off_rb_pay = take(rrec * 4);   // 16 bytes per visible record, list order
  P->off_rb_spay = take(rrec * 4);  // the same in depth order
  P->off_rb_zrec = take(rrec);      // depth bits by record id
  P->ws_size = o;
  P->magic = kPlanMagic;
  return GS_OK;
}

size_t gs_workspace_size(const gs_plan* plan) {
  if (check_plan(plan) != GS_OK) return 0;
  return plan_of(plan)->ws_size;
}

int64_t gs_plan_total_pixels(const gs_plan* plan) {
  if (check_plan(plan) != GS_OK) return -1;
  return plan_of(plan)->vt.total_pix;
}

int64_t gs_plan_pixel_offset(const gs_plan* plan, int32_t view) {
  if (check_plan(plan) != GS_OK) return -1;
  const Plan* P = plan_of(plan);
  if (view < 0 || view >= P->n_views) return -1;
  return P->vt.v[view].pix_off;
}

int64_t gs_plan_total_tiles(const gs_plan* plan) {
  if (check_plan(plan) != GS_OK) return -1;
  return plan_of(plan)->vt.total_tiles;
}

int64_t gs_plan_ws_offset(const gs_plan* plan, int32_t region) {
  if (check_plan(plan) != GS_OK) return -1;
  const Plan& P = *plan_of(plan);
  switch (region) {
    case GS_WS_RECORDS: return (int64_t)P.off_rec;
    case GS_WS_RECTS: return (int64_t)P.off_rect;
    case GS_WS_TILES_TOUCHED: return (int64_t)P.off_tt;
    case GS_WS_PAIR_OFFSETS: return (int64_t)P.off_poff;
    case GS_WS_SORTED_KEYS: return (int64_t)P.off_keys;
    case GS_WS_SORTED_VALS: return (int64_t)P.off_vals;
    case GS_WS_SORTED_RECS: return (int64_t)P.off_sorted_rec;
    case GS_WS_RANGES: return (int64_t)P.off_ranges;
    default: return -1;
  }
}

int32_t* gs_flags_ptr(const gs_plan* plan, void* ws) {
  if (check_plan(plan) != GS_OK || !ws) return nullptr;
  return ws_at<int32_t>(ws, plan_of(plan)->off_flags);
}

// Preprocess.  clear: the per-iteration flags and the per-tile pair
// counters are zeroed by a kernel first (graph-safe); a whole iteration
// skips it, the binning of the previous one having left them zero.
static gs_status preprocess_enqueue(const gs_plan* plan, const gs_gaussians* g,
                                    const float* cams_dev, void* ws, hipStream_t s, bool clear) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_ws(P, ws)) != GS_OK) return st;
  if ((st = check_gaussians(P, g)) != GS_OK) return st;
  if (!cams_dev) return fail(GS_ERR_INVALID_ARG, "cams_dev is null");
  hipError_t e = clear ? launch_clear_counters(P, ws, s) : hipSuccess;
  if (e == hipSuccess) e = launch_preprocess(P, *g, cams_dev, ws, s);
  return hip_check(e, "gs_preprocess");
}

gs_status gs_preprocess(const gs_plan* plan, const gs_gaussians* g, const float* cams_dev,
                        void* ws, void* stream) {
  return preprocess_enqueue(plan, g, cams_dev, ws, static_cast<hipStream_t>(stream), true);
}

gs_status gs_bin_sort(const gs_plan* plan, void* ws, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_ws(P, ws)) != GS_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_bin_sort(P, ws, s);
  return hip_check(e, "gs_bin_sort");
}

static int persistent_grid(const Plan& P, bool bwd) {
  const int per_cu = render_blocks_per_cu(P, bwd);
  const int64_t items = (P.vt.total_tiles + P.cfg.chunk - 1) / P.cfg.chunk;
  return (int)std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)device_cus() * per_cu));
}

gs_status gs_render_fwd(const gs_plan* plan, void* ws, const float* cams_dev, float* color,
                        float* depth, float* T_final, uint32_t* last, const float* target_rgb,
                        const float* target_depth, float* loss_per_view, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_ws(P, ws)) != GS_OK) return st;
  if (!cams_dev) return fail(GS_ERR_INVALID_ARG, "cams_dev is null");
  if (!color || !depth || !T_final || !last) return fail(GS_ERR_INVALID_ARG, "output image pointer is null");
  if (target_rgb && !loss_per_view) return fail(GS_ERR_INVALID_ARG, "target_rgb given without loss_per_view");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool pers = (P.cfg.flags & GS_PERSISTENT) != 0;
  int32_t* fl = ws_at<int32_t>(ws, P.off_flags);
  hipError_t e = hipSuccess;
  if (e == hipSuccess)
    e = launch_render_fwd(P, ws, cams_dev, color, depth, T_final, last, target_rgb, target_depth,
                          loss_per_view, ws_at<uint32_t>(ws, P.off_order),
                          pers ? fl + F_QUEUE_FWD : nullptr,
                          pers ? persistent_grid(P, false) : P.vt.total_tiles, s);
  return hip_check(e, "gs_render_fwd");
}

}  // extern "C"

extern "C" {

gs_status gs_render_bwd_raster(const gs_plan* plan, void* ws, const float* cams_dev,
                               const float* color, const float* depth, const float* T_final,
                               const uint32_t* last, const float* dL_dcolor,
                               const float* dL_ddepth, const float* target_rgb,
                               const float* target_depth, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_ws(P, ws)) != GS_OK) return st;
  if (!cams_dev) return fail(GS_ERR_INVALID_ARG, "cams_dev is null");
  if (!color || !depth || !T_final || !last) return fail(GS_ERR_INVALID_ARG, "forward buffers must be non-null");
  const bool fused = (P.cfg.flags & GS_FUSED_L1) != 0;
  if (fused && !target_rgb) return fail(GS_ERR_INVALID_ARG, "GS_FUSED_L1 needs target_rgb");
  if (!fused && !dL_dcolor) return fail(GS_ERR_INVALID_ARG, "dL_dcolor is null (and GS_FUSED_L1 not set)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool splat = (P.cfg.flags & GS_SPLAT_BWD) != 0;
  const bool pers = !splat && (P.cfg.flags & GS_PERSISTENT) != 0;
  int32_t* fl = ws_at<int32_t>(ws, P.off_flags);
  hipError_t e = hipSuccess;
  // splat-wise: grid-stride over the buckets, as many waves as stay resident
  const int grid = splat ? (int)std::max<int64_t>(1, std::min<int64_t>(P.ckpt_slots, (int64_t)device_cus() * splat_blocks_per_cu(P)))
                         : (pers ? persistent_grid(P, true) : P.vt.total_tiles);
  if (e == hipSuccess)
    e = launch_render_bwd(P, ws, cams_dev, color, depth, T_final, last, dL_dcolor, dL_ddepth,
                          target_rgb, target_depth, fused ? 1 : 0, sorted_vals(P, ws),
                          ws_at<uint32_t>(ws, P.off_order),
                          pers ? fl + F_QUEUE_BWD : nullptr, grid, s);
  return hip_check(e, "gs_render_bwd_raster");
}

gs_status gs_project_bwd(const gs_plan* plan, const gs_gaussians* g, const float* cams_dev,
                         void* ws, const gs_gaussian_grads* out, float* dL_dpose, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_ws(P, ws)) != GS_OK) return st;
  if ((st = check_gaussians(P, g)) != GS_OK) return st;
  if (!cams_dev) return fail(GS_ERR_INVALID_ARG, "cams_dev is null");
  if (!out || (P.n > 0 && (!out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh)))
    return fail(GS_ERR_INVALID_ARG, "gradient output pointers must be non-null");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return hip_check(launch_project_bwd(P, *g, cams_dev, ws, *out, dL_dpose,
                                      (P.cfg.flags & GS_ACCUMULATE_GRADS) ? 1 : 0, false, s),
                   "gs_project_bwd");
}

gs_status gs_render_bwd(const gs_plan* plan, const gs_gaussians* g, const float* cams_dev,
                        void* ws, const float* color, const float* depth,
                        const float* T_final, const uint32_t* last,
                        const float* dL_dcolor, const float* dL_ddepth,
                        const float* target_rgb, const float* target_depth,
                        const gs_gaussian_grads* out, float* dL_dpose, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_gaussians(P, g)) != GS_OK) return st;
  if (!out || (P.n > 0 && (!out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh)))
    return fail(GS_ERR_INVALID_ARG, "gradient output pointers must be non-null");
  st = gs_render_bwd_raster(plan, ws, cams_dev, color, depth, T_final, last, dL_dcolor,
                            dL_ddepth, target_rgb, target_depth, stream);
  if (st != GS_OK) return st;
  return gs_project_bwd(plan, g, cams_dev, ws, out, dL_dpose, stream);
}

gs_status gs_render_loss(const gs_plan* plan, void* ws, const float* color, const float* depth,
                         const float* target_rgb, const float* target_depth, double lambda_ssim,
                         float* dL_dcolor, float* dL_ddepth, float* loss_per_view, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_ws(P, ws)) != GS_OK) return st;
  if (!color || !depth || !target_rgb || !dL_dcolor || !dL_ddepth)
    return fail(GS_ERR_INVALID_ARG, "color, depth, target_rgb, dL_dcolor and dL_ddepth must be non-null");
  if (!(lambda_ssim >= 0.0 && lambda_ssim <= 1.0)) return fail(GS_ERR_INVALID_ARG, "lambda_ssim must be in [0, 1]");
  return hip_check(launch_render_loss(P, ws, color, depth, target_rgb, target_depth, lambda_ssim,
                                      dL_dcolor, dL_ddepth, loss_per_view,
                                      static_cast<hipStream_t>(stream)),
                   "gs_render_loss");
}

static gs_status check_adam(const gs_param_group* groups, int32_t n_groups, int32_t step,
                            double beta1, double beta2, double eps, const int32_t* step_dev) {
  if (n_groups < 0 || (n_groups > 0 && !groups)) return fail(GS_ERR_INVALID_ARG, "bad group array");
  if (!step_dev && step < 1) return fail(GS_ERR_INVALID_ARG, "step must be >= 1");
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0))
    return fail(GS_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  for (int k = 0; k < n_groups; ++k) {
    const gs_param_group& G = groups[k];
    if (G.n < 0) return fail(GS_ERR_INVALID_ARG, "group %d: n < 0", k);
    if (G.n > 0 && (!G.p || !G.g || !G.m || !G.v)) return fail(GS_ERR_INVALID_ARG, "group %d: null pointer", k);
    if (!aligned(G.p, 16) || !aligned(G.g, 16) || !aligned(G.m, 16) || !aligned(G.v, 16))
      return fail(GS_ERR_INVALID_ARG, "group %d: pointers must be 16-byte aligned", k);
  }
  return GS_OK;
}

gs_status gs_adam_step(const gs_param_group* groups, int32_t n_groups, int32_t step,
                       double beta1, double beta2, double eps, double lambda_o,
                       int64_t reg_count, int32_t* step_dev, void* stream) {
  gs_status st = check_adam(groups, n_groups, step, beta1, beta2, eps, step_dev);
  if (st != GS_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return hip_check(launch_adam(groups, n_groups, step, beta1, beta2, eps, lambda_o, reg_count,
                               step_dev, s),
                   "gs_adam_step");
}

size_t gs_spatial_order_tmp_bytes(int64_t n) { return spatial_order_tmp_bytes(n); }

gs_status gs_spatial_order(const float* means, int64_t n, int32_t* perm, void* tmp, void* stream) {
  if (n < 0 || n > INT32_MAX) return fail(GS_ERR_INVALID_ARG, "n must be 0..2^31-1");
  if (n == 0) return GS_OK;
  if (!means || !perm || !tmp) return fail(GS_ERR_INVALID_ARG, "null pointer");
  if (!aligned(tmp, 256)) return fail(GS_ERR_INVALID_ARG, "tmp must be 256-byte aligned");
  return hip_check(launch_spatial_order(means, n, perm, tmp, static_cast<hipStream_t>(stream)),
                   "gs_spatial_order");
}

gs_status gs_permute_gaussians(const gs_gaussians* src, const int32_t* perm,
                               const gs_gaussian_grads* dst, void* stream) {
  if (!src || !dst || (src->n > 0 && !perm)) return fail(GS_ERR_INVALID_ARG, "null argument");
  if (src->n < 0 || src->n > INT32_MAX) return fail(GS_ERR_INVALID_ARG, "n must be 0..2^31-1");
  if (src->sh_degree < 0 || src->sh_degree > 3) return fail(GS_ERR_UNSUPPORTED, "sh_degree must be 0..3");
  if (src->n == 0) return GS_OK;
  if (!src->means || !src->log_scales || !src->quats || !src->opacity_logits || !src->sh ||
      !dst->means || !dst->log_scales || !dst->quats || !dst->opacity_logits || !dst->sh)
    return fail(GS_ERR_INVALID_ARG, "null parameter pointer");
  const int K3 = 3 * (src->sh_degree + 1) * (src->sh_degree + 1);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_gather_rows(src->means, perm, src->n, 3, dst->means, s);
  if (e == hipSuccess) e = launch_gather_rows(src->log_scales, perm, src->n, 3, dst->log_scales, s);
  if (e == hipSuccess) e = launch_gather_rows(src->quats, perm, src->n, 4, dst->quats, s);
  if (e == hipSuccess) e = launch_gather_rows(src->opacity_logits, perm, src->n, 1, dst->opacity_logits, s);
  if (e == hipSuccess) e = launch_gather_rows(src->sh, perm, src->n, K3, dst->sh, s);
  return hip_check(e, "gs_permute_gaussians");
}

gs_status gs_pose_retract(const float* cams_in, const float* xi, float* cams_out,
                          int32_t n_views, void* stream) {
  if (n_views < 1 || n_views > GS_MAX_VIEWS) return fail(GS_ERR_INVALID_ARG, "n_views must be 1..%d", GS_MAX_VIEWS);
  if (!cams_in || !xi || !cams_out) return fail(GS_ERR_INVALID_ARG, "null pointer");
  return hip_check(launch_pose_retract(cams_in, xi, cams_out, n_views,
                                       static_cast<hipStream_t>(stream)),
                   "gs_pose_retract");
}

gs_status gs_pose_tangent_vjp(const float* xi, const float* dL_ddelta, float* dL_dxi,
                              int32_t n_views, void* stream) {
  if (n_views < 1 || n_views > GS_MAX_VIEWS) return fail(GS_ERR_INVALID_ARG, "n_views must be 1..%d", GS_MAX_VIEWS);
  if (!xi || !dL_ddelta || !dL_dxi) return fail(GS_ERR_INVALID_ARG, "null pointer");
  return hip_check(launch_pose_vjp(xi, dL_ddelta, dL_dxi, n_views, static_cast<hipStream_t>(stream)),
                   "gs_pose_tangent_vjp");
}

gs_status gs_grad_stats(const gs_plan* plan, void* ws, float* accum, float* denom, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_ws(P, ws)) != GS_OK) return st;
  if (P.n > 0 && (!accum || !denom)) return fail(GS_ERR_INVALID_ARG, "accum and denom must be non-null");
  return hip_check(launch_grad_stats(P, ws, accum, denom, static_cast<hipStream_t>(stream)),
                   "gs_grad_stats");
}

size_t gs_densify_tmp_bytes(int64_t n) { return n < 0 ? 0 : densify_tmp_bytes(n); }

static bool grads_ok(const gs_gaussian_grads* x) {
  return x && x->means && x->log_scales && x->quats && x->opacity_logits && x->sh;
}

gs_status gs_densify_prune(const gs_gaussians* g, const gs_gaussian_grads* m,
                           const gs_gaussian_grads* v, const float* accum, const float* denom,
                           const float* normals, float tau_p, float eps_alpha,
                           float percent_dense, float extent, const gs_gaussian_grads* out,
                           const gs_gaussian_grads* out_m, const gs_gaussian_grads* out_v,
                           int64_t out_capacity, int32_t* n_out, void* tmp, void* stream) {
  if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return fail(GS_ERR_INVALID_ARG, "bad gaussians");
  if (g->n > INT32_MAX / 2) return fail(GS_ERR_INVALID_ARG, "too many Gaussians");
  if (!n_out || !tmp || !aligned(tmp, 256)) return fail(GS_ERR_INVALID_ARG, "n_out and a 256-byte aligned tmp are required");
  if (out_capacity < 0) return fail(GS_ERR_INVALID_ARG, "out_capacity < 0");
  if (g->n > 0) {
    if (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh || !accum || !denom ||
        !normals || !grads_ok(m) || !grads_ok(v) || !grads_ok(out) || !grads_ok(out_m) || !grads_ok(out_v))
      return fail(GS_ERR_INVALID_ARG, "null pointer");
  }
  if (!(tau_p >= 0.0f && eps_alpha >= 0.0f && percent_dense >= 0.0f && extent >= 0.0f))
    return fail(GS_ERR_INVALID_ARG, "thresholds must be >= 0");
  return hip_check(launch_densify(*g, *m, *v, accum, denom, normals, tau_p, eps_alpha,
                                  percent_dense, extent, *out, *out_m, *out_v, out_capacity,
                                  n_out, tmp, static_cast<hipStream_t>(stream)),
                   "gs_densify_prune");
}

}  // extern "C"

namespace {

// Scratch of the stand-alone sort for n pairs: second key and value buffers,
// the per-block digit histograms, the digit totals and the pair count.
struct SortTmp {
  size_t k1, v1, hist, dtot, cnt, bytes;
};

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

constexpr SortTmp sort_tmp_layout(int64_t n) {
  const int64_t nb = n > kSortTile ? (n + kSortTile - 1) / kSortTile : 1;
  SortTmp t{};
  t.k1 = 0;
  t.v1 = align256(t.k1 + (size_t)n * 8 + 8);
  t.hist = align256(t.v1 + (size_t)n * 4 + 4);
  t.dtot = align256(t.hist + (size_t)kRadix * nb * 4);
  t.cnt = align256(t.dtot + kRadix * 4);
  t.bytes = align256(t.cnt + 16);
  return t;
}

// Sort with caller-provided scratch `tmp` (sort_tmp_layout(n).bytes, 256-byte
// aligned); n >= 1 and the arguments already checked.
gs_status sort_pairs_in(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits, void* tmp,
                        hipStream_t s, const char* what) {
  const int64_t nb = std::max<int64_t>(1, (n + kSortTile - 1) / kSortTile);
  const SortTmp L = sort_tmp_layout(n);
  char* base = static_cast<char*>(tmp);
  uint64_t* k1 = reinterpret_cast<uint64_t*>(base + L.k1);
  uint32_t* v1 = reinterpret_cast<uint32_t*>(base + L.v1);
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + L.hist);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(base + L.dtot);
  int32_t* cnt = reinterpret_cast<int32_t*>(base + L.cnt);
  // the pair count is written by a kernel on every call, every histogram
  // entry the passes read is written by the same call: nothing in the
  // scratch has to start at zero
  hipError_t e = launch_set_i32(cnt, (int32_t)n, s);
  int which = 0;
  if (e == hipSuccess)
    e = launch_radix_sort(keys, k1, vals, v1, cnt, hist, dtot, nb, key_bits, false, &which, s);
  if (e == hipSuccess && which == 1) {
    e = hipMemcpyAsync(keys, k1, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(vals, v1, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
  }
  return hip_check(e, what);
}

gs_status check_sort_args(const uint64_t* keys, const uint32_t* vals, int64_t n, int64_t n_max,
                          int32_t key_bits) {
  if (n < 0 || n > n_max) return fail(GS_ERR_INVALID_ARG, "n must be 0..%lld", (long long)n_max);
  if (key_bits < 1 || key_bits > 64) return fail(GS_ERR_INVALID_ARG, "key_bits must be 1..64");
  if (n > 0 && (!keys || !vals)) return fail(GS_ERR_INVALID_ARG, "null pointer");
  return GS_OK;
}

// Allocation-free variant: the scratch of GS_SORT_NOALLOC_MAX pairs is a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes the array's own name to a kernel or a copy (on the
// host it is only a stand-in for the symbol): each device's address comes
// from hipGetSymbolAddress, taken once per device with that device current.
constexpr SortTmp kNoallocLayout = sort_tmp_layout(GS_SORT_NOALLOC_MAX);
static __device__ __align__(256) unsigned char scratch[kNoallocLayout.bytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gs_status scratch_of_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(e, "gs_sort_pairs_noalloc (hipGetDevice)");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(GS_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "gs_sort_pairs_noalloc (hipGetSymbolAddress)");
    if (!p || !aligned(p, 256))
      return fail(GS_ERR_HIP, "gs_sort_pairs_noalloc: bad scratch address on device %d", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace

extern "C" {

size_t gs_sort_tmp_bytes(int64_t n) {
  if (n < 0) return 0;
  return sort_tmp_layout(n).bytes;
}

gs_status gs_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits, void* tmp,
                        void* stream) {
  gs_status st = check_sort_args(keys, vals, n, INT32_MAX, key_bits);
  if (st != GS_OK || n == 0) return st;
  if (!tmp) return fail(GS_ERR_INVALID_ARG, "null pointer");
  if (!aligned(tmp, 256)) return fail(GS_ERR_INVALID_ARG, "tmp must be 256-byte aligned");
  return sort_pairs_in(keys, vals, n, key_bits, tmp, static_cast<hipStream_t>(stream),
                       "gs_sort_pairs");
}

gs_status gs_sort_pairs_noalloc(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits,
                                void* stream) {
  gs_status st = check_sort_args(keys, vals, n, GS_SORT_NOALLOC_MAX, key_bits);
  if (st != GS_OK || n == 0) return st;
  void* tmp = nullptr;
  if ((st = scratch_of_current_device(&tmp)) != GS_OK) return st;
  return sort_pairs_in(keys, vals, n, key_bits, tmp, static_cast<hipStream_t>(stream),
                       "gs_sort_pairs_noalloc");
}

static gs_status check_gather(const Plan& P, const gs_view_gather* g, const float* cams_out,
                              const float* rgb_out, const float* depth_out) {
  if (!g || !g->pool_cams || !g->pool_rgb || !g->sel)
    return fail(GS_ERR_INVALID_ARG, "gather: null pool or selection pointer");
  if (g->n_pool < 1) return fail(GS_ERR_INVALID_ARG, "gather: n_pool must be >= 1");
  if (!cams_out || !rgb_out) return fail(GS_ERR_INVALID_ARG, "gather: null camera or colour slots");
  if ((g->pool_depth != nullptr) != (depth_out != nullptr))
    return fail(GS_ERR_INVALID_ARG, "gather: depth pool and depth slots go together");
  for (int v = 1; v < P.vt.n_views; ++v)
    if (P.vt.v[v].W != P.vt.v[0].W || P.vt.v[v].H != P.vt.v[0].H)
      return fail(GS_ERR_INVALID_ARG, "gather: every view must have the keyframes' size");
  return GS_OK;
}

gs_status gs_gather_views(const gs_plan* plan, const gs_view_gather* g, float* cams_out,
                          float* rgb_out, float* depth_out, void* stream) {
  gs_status st;
  if ((st = check_plan(plan)) != GS_OK) return st;
  const Plan& P = *plan_of(plan);
  if ((st = check_gather(P, g, cams_out, rgb_out, depth_out)) != GS_OK) return st;
  return hip_check(launch_gather_views(P, *g, cams_out, rgb_out, depth_out,
                                       static_cast<hipStream_t>(stream)),
                   "gs_gather_views");
}

}  // extern "C"

// One mapping iteration; `marks` (optional) records the timing events of
// gs_iteration_time_marks between the launches.
static gs_status iteration_enqueue(const gs_iteration* it, void* stream, const Marks* marks) {
  const Marks none{};
  const Marks& mk = marks ? *marks : none;
  if (!it) return fail(GS_ERR_INVALID_ARG, "iteration is null");
  if (!it->plan || check_plan(it->plan) != GS_OK) return fail(GS_ERR_INVALID_ARG, "bad plan");
  if (it->n_adam_groups < 0 || (it->n_adam_groups > 0 && !it->adam_groups))
    return fail(GS_ERR_INVALID_ARG, "bad Adam group array");
  if (it->n_adam_groups > 0 && !it->step_dev)
    return fail(GS_ERR_INVALID_ARG, "an iteration with Adam needs step_dev (the device step counter)");
  const Plan& P = *plan_of(it->plan);
  const bool ssim = it->lambda_ssim > 0.0;
  if (ssim) {
    if (!(it->lambda_ssim <= 1.0)) return fail(GS_ERR_INVALID_ARG, "lambda_ssim must be in [0, 1]");
    if (P.cfg.flags & GS_FUSED_L1)
      return fail(GS_ERR_INVALID_ARG, "lambda_ssim > 0 takes explicit loss gradients: clear GS_FUSED_L1");
    if (!it->target_rgb || !it->loss_grad_color || !it->loss_grad_depth)
      return fail(GS_ERR_INVALID_ARG, "lambda_ssim > 0 needs target_rgb and loss gradient buffers");
  }
  if (it->gather) {
    gs_status st = check_gather(P, it->gather, it->cams_dev, it->target_rgb, it->target_depth);
    if (st != GS_OK) return st;
  }
  // the scheduled keyframes into the batch slots, before anything reads them
  auto gather = [&]() -> gs_status {
    if (!it->gather) return GS_OK;
    return hip_check(launch_gather_views(P, *it->gather, const_cast<float*>(it->cams_dev),
                                         const_cast<float*>(it->target_rgb),
                                         const_cast<float*>(it->target_depth),
                                         static_cast<hipStream_t>(stream)),
                     "gs_iteration_enqueue (gather)");
  };
  // One view with Adam: the projection backward writes the gradients of the
  // Gaussians with pairs only, and Adam takes the others as zero (no zero
  // fill, no read).  The gradient buffers are left unspecified for those.
  const bool sparse = it->n_adam_groups > 0 && it->n_adam_groups <= kAdamFoldGroups && P.vt.n_views == 1 &&
                      !(P.cfg.flags & GS_ACCUMULATE_GRADS) && P.n > 0;
  hipStream_t strm = static_cast<hipStream_t>(stream);
  if (!sparse) {
    gs_status st = gather();
    if (st != GS_OK) return st;
    if ((st = hip_check(mk.at(GS_MARK_START, strm), "timing mark")) != GS_OK) return st;
    st = gs_preprocess(it->plan, &it->gaussians, it->cams_dev, it->ws, stream);
    if (st != GS_OK) return st;
    if ((st = hip_check(mk.at(GS_MARK_PREPROCESS, strm), "timing mark")) != GS_OK) return st;
    if ((st = check_ws(P, it->ws)) != GS_OK) return st;
    st = hip_check(launch_bin_sort(P, it->ws, strm, false, nullptr, marks), "gs_bin_sort");
    if (st != GS_OK) return st;
    st = gs_render_fwd(it->plan, it->ws, it->cams_dev, it->color, it->depth, it->T_final, it->last,
                       ssim ? nullptr : it->target_rgb, ssim ? nullptr : it->target_depth,
                       ssim ? nullptr : it->loss_per_view, stream);
    if (st != GS_OK) return st;
    if ((st = hip_check(mk.at(GS_MARK_FORWARD, strm), "timing mark")) != GS_OK) return st;
    const float* gC = it->dL_dcolor;
    const float* gD = it->dL_ddepth;
    if (ssim) {
      st = gs_render_loss(it->plan, it->ws, it->color, it->depth, it->target_rgb, it->target_depth,
                          it->lambda_ssim, it->loss_grad_color, it->loss_grad_depth,
                          it->loss_per_view, stream);
      if (st != GS_OK) return st;
      gC = it->loss_grad_color;
      gD = it->loss_grad_depth;
    }
    if ((st = hip_check(mk.at(GS_MARK_LOSS, strm), "timing mark")) != GS_OK) return st;
    // gs_render_bwd as its two halves, with a mark between them
    if ((st = check_gaussians(P, &it->gaussians)) != GS_OK) return st;
    const gs_gaussian_grads* out = &it->grads;
    if (P.n > 0 && (!out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh))
      return fail(GS_ERR_INVALID_ARG, "gradient output pointers must be non-null");
    st = gs_render_bwd_raster(it->plan, it->ws, it->cams_dev, it->color, it->depth, it->T_final,
                              it->last, gC, gD, it->target_rgb, it->target_depth, stream);
    if (st != GS_OK) return st;
    if ((st = hip_check(mk.at(GS_MARK_RASTER_BWD, strm), "timing mark")) != GS_OK) return st;
    st = gs_project_bwd(it->plan, &it->gaussians, it->cams_dev, it->ws, out, it->dL_dpose, stream);
    if (st != GS_OK) return st;
    if ((st = hip_check(mk.at(GS_MARK_PROJECT_BWD, strm), "timing mark")) != GS_OK) return st;
    if (it->n_adam_groups > 0) {
      // the Adam launch (and the step advance after it) do nothing when the
      // binning of this iteration overflowed
      st = check_adam(it->adam_groups, it->n_adam_groups, 1, it->beta1, it->beta2, it->eps,
                      it->step_dev);
      if (st != GS_OK) return st;
      st = hip_check(launch_adam(it->adam_groups, it->n_adam_groups, 1, it->beta1, it->beta2,
                                 it->eps, it->lambda_o, it->reg_count, it->step_dev,
                                 static_cast<hipStream_t>(stream), nullptr, nullptr,
                                 ws_at<int32_t>(it->ws, P.off_flags) + F_OVERFLOW),
                     "gs_iteration_enqueue (Adam)");
      if (st != GS_OK) return st;
    }
    return hip_check(mk.at(GS_MARK_ADAM, strm), "timing mark");
  }

  // Sparse path: everything is checked before anything is enqueued.
  gs_status st;
  if ((st = check_ws(P, it->ws)) != GS_OK) return st;
  if ((st = check_gaussians(P, &it->gaussians)) != GS_OK) return st;
  if (!it->cams_dev) return fail(GS_ERR_INVALID_ARG, "cams_dev is null");
  if (!it->color || !it->depth || !it->T_final || !it->last)
    return fail(GS_ERR_INVALID_ARG, "output image pointer is null");
  if (!ssim && it->target_rgb && !it->loss_per_view)
    return fail(GS_ERR_INVALID_ARG, "target_rgb given without loss_per_view");
  const bool fused = (P.cfg.flags & GS_FUSED_L1) != 0;
  if (!ssim && fused && !it->target_rgb) return fail(GS_ERR_INVALID_ARG, "GS_FUSED_L1 needs target_rgb");
  if (!ssim && !fused && !it->dL_dcolor)
    return fail(GS_ERR_INVALID_ARG, "dL_dcolor is null (and GS_FUSED_L1 not set)");
  const gs_gaussian_grads& gr = it->grads;
  if (!gr.means || !gr.log_scales || !gr.quats || !gr.opacity_logits || !gr.sh)
    return fail(GS_ERR_INVALID_ARG, "gradient output pointers must be non-null");
  if (!(it->beta1 >= 0.0 && it->beta1 < 1.0 && it->beta2 >= 0.0 && it->beta2 < 1.0 && it->eps >= 0.0))
    return fail(GS_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  int64_t adam_elems = 0;
  for (int k = 0; k < it->n_adam_groups; ++k) {
    const gs_param_group& G = it->adam_groups[k];
    if (G.n < 0) return fail(GS_ERR_INVALID_ARG, "group %d: negative size", k);
    if (G.n > 0 && (!G.p || !G.g || !G.m || !G.v)) return fail(GS_ERR_INVALID_ARG, "group %d: null pointer", k);
    if (!aligned(G.p, 16) || !aligned(G.g, 16) || !aligned(G.m, 16) || !aligned(G.v, 16))
      return fail(GS_ERR_INVALID_ARG, "group %d: pointers must be 16-byte aligned", k);
    adam_elems += G.n;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // The Adam step counter is advanced by the binning scan of the iteration
  // and the one-view loss reduction rides on the Adam launch: two launches
  // fewer per iteration, same values.
  AdamFold fold{};
  fold.step_taken = it->step_dev != nullptr;
  AdamStepFactors* factors =
      reinterpret_cast<AdamStepFactors*>(ws_at<char>(it->ws, P.off_flags) + kBiasOffset);
  fold.factors = factors;
  StepAdvance adv{};
  adv.step = it->step_dev;
  adv.beta1 = it->beta1;
  adv.beta2 = it->beta2;
  adv.out = factors;
  adv.n_groups = it->n_adam_groups;
  for (int k = 0; k < it->n_adam_groups; ++k) adv.lr[k] = it->adam_groups[k].lr;
  const bool fold_loss = !ssim && it->target_rgb && adam_elems > 0;
  if (fold_loss) {
    const ViewInfo& vi = P.vt.v[0];
    fold.tile_loss = ws_at<float2>(it->ws, P.off_tile_loss) + vi.tile_off;
    fold.loss_tiles = vi.tiles_x * vi.tiles_y;
    fold.loss_has_depth = it->target_depth ? 1 : 0;
    fold.loss_pixels = (double)vi.W * vi.H;
    fold.lambda_depth = P.cfg.lambda_depth;
    fold.loss = it->loss_per_view;
  }
  // no clearing launch: the counters were left zero by the last binning on
  // this workspace (or the workspace is fresh, zero-filled)
  if ((st = gather()) != GS_OK) return st;
  if ((st = hip_check(mk.at(GS_MARK_START, s), "timing mark")) != GS_OK) return st;
  st = preprocess_enqueue(it->plan, &it->gaussians, it->cams_dev, it->ws, s, false);
  if (st != GS_OK) return st;
  if ((st = hip_check(mk.at(GS_MARK_PREPROCESS, s), "timing mark")) != GS_OK) return st;
  // the binning leaves the short lists to the forward, which sorts each
  // tile's list right before compositing it (one launch fewer; the sort's
  // memory latency hides behind other wavefronts' compositing); its scan
  // advances the Adam step unless the pairs overflow
  hipError_t e = launch_bin_sort(P, it->ws, s, true, it->step_dev ? &adv : nullptr, marks);
  TileSortArgs fwd_sort = tile_sort_args(P, it->ws);
  fwd_sort.long_after = false;  // the long lists were sorted by the binning
  if (e != hipSuccess) return hip_check(e, "gs_iteration_enqueue (binning)");
  const bool pers = (P.cfg.flags & GS_PERSISTENT) != 0;
  int32_t* fl = ws_at<int32_t>(it->ws, P.off_flags);
  e = launch_render_fwd(
      P, it->ws, it->cams_dev, it->color, it->depth, it->T_final, it->last,
      ssim ? nullptr : it->target_rgb, ssim ? nullptr : it->target_depth,
      (ssim || fold_loss) ? nullptr : it->loss_per_view,
      ws_at<uint32_t>(it->ws, P.off_order), pers ? fl + F_QUEUE_FWD : nullptr,
      pers ? persistent_grid(P, false) : P.vt.total_tiles, s, fwd_sort);
  if (e == hipSuccess) e = mk.at(GS_MARK_FORWARD, s);
  if (e != hipSuccess) return hip_check(e, "gs_iteration_enqueue (forward)");
  const float* gC = it->dL_dcolor;
  const float* gD = it->dL_ddepth;
  if (ssim) {
    st = gs_render_loss(it->plan, it->ws, it->color, it->depth, it->target_rgb, it->target_depth,
                        it->lambda_ssim, it->loss_grad_color, it->loss_grad_depth,
                        it->loss_per_view, stream);
    if (st != GS_OK) return st;
    gC = it->loss_grad_color;
    gD = it->loss_grad_depth;
  }
  if ((st = hip_check(mk.at(GS_MARK_LOSS, s), "timing mark")) != GS_OK) return st;
  st = gs_render_bwd_raster(it->plan, it->ws, it->cams_dev, it->color, it->depth, it->T_final,
                            it->last, gC, gD, it->target_rgb, it->target_depth, stream);
  if (st != GS_OK) return st;
  if ((st = hip_check(mk.at(GS_MARK_RASTER_BWD, s), "timing mark")) != GS_OK) return st;
  e = launch_project_bwd(P, it->gaussians, it->cams_dev, it->ws, gr, it->dL_dpose, 0, true, s);
  if (e == hipSuccess) e = mk.at(GS_MARK_PROJECT_BWD, s);
  if (e != hipSuccess) return hip_check(e, "gs_iteration_enqueue (projection backward)");
  const uint32_t* vis[16];
  int32_t per[16];
  const uint32_t* tt = ws_at<uint32_t>(it->ws, P.off_tt);
  for (int k = 0; k < it->n_adam_groups; ++k) {
    const float* g = it->adam_groups[k].g;
    vis[k] = tt;
    if (g == gr.means || g == gr.log_scales) per[k] = 3;
    else if (g == gr.quats) per[k] = 4;
    else if (g == gr.opacity_logits) per[k] = 1;
    else if (g == gr.sh) per[k] = 3 * P.K;
    else per[k] = 0;
    if (per[k] == 0 || it->adam_groups[k].n != (int64_t)per[k] * P.n) {
      vis[k] = nullptr;  // not (all of) a gradient this iteration writes: read as is
      per[k] = 1;
    }
  }
  e = launch_adam(it->adam_groups, it->n_adam_groups, 1, it->beta1, it->beta2, it->eps,
                  it->lambda_o, it->reg_count, it->step_dev, s, vis, per,
                  ws_at<int32_t>(it->ws, P.off_flags) + F_OVERFLOW, &fold);
  if (e == hipSuccess) e = mk.at(GS_MARK_ADAM, s);
  return hip_check(e, "gs_iteration_enqueue (Adam)");
}

extern "C" {

gs_status gs_iteration_enqueue(const gs_iteration* it, void* stream) {
  return iteration_enqueue(it, stream, nullptr);
}

gs_status gs_iteration_time_marks(const gs_iteration* it, void* stream, int32_t warmup,
                                  int32_t reps, float* ms) {
  if (!it || !ms || warmup < 0 || reps < 1)
    return fail(GS_ERR_INVALID_ARG, "bad gs_iteration_time_marks arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cap);
  if (e != hipSuccess) return hip_check(e, "gs_iteration_time_marks");
  if (cap != hipStreamCaptureStatusNone)
    return fail(GS_ERR_INVALID_ARG, "gs_iteration_time_marks cannot run under stream capture");
  gs_status st = GS_OK;
  for (int i = 0; st == GS_OK && i < warmup; ++i) st = iteration_enqueue(it, stream, nullptr);
  if (st != GS_OK) return st;
  std::vector<hipEvent_t> ev((size_t)reps * GS_N_MARKS, nullptr);
  for (size_t k = 0; e == hipSuccess && k < ev.size(); ++k) e = hipEventCreate(&ev[k]);
  for (int r = 0; e == hipSuccess && st == GS_OK && r < reps; ++r) {
    Marks m;
    m.ev = ev.data() + (size_t)r * GS_N_MARKS;
    st = iteration_enqueue(it, stream, &m);
  }
  if (e == hipSuccess && st == GS_OK) e = hipStreamSynchronize(s);
  for (int r = 0; e == hipSuccess && st == GS_OK && r < reps; ++r)
    for (int k = 0; e == hipSuccess && k + 1 < GS_N_MARKS; ++k) {
      float t = 0.0f;
      e = hipEventElapsedTime(&t, ev[(size_t)r * GS_N_MARKS + k], ev[(size_t)r * GS_N_MARKS + k + 1]);
      ms[(size_t)r * (GS_N_MARKS - 1) + k] = t;
    }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st != GS_OK) return st;
  return hip_check(e, "gs_iteration_time_marks");
}

struct gs_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

gs_status gs_graph_create(const gs_iteration* it, void* stream, gs_graph** out) {
  if (!it || !out) return fail(GS_ERR_INVALID_ARG, "null argument");
  if (!stream) return fail(GS_ERR_INVALID_ARG, "graph capture needs a non-null stream");
  if (it->n_adam_groups > 0 && !it->step_dev)
    return fail(GS_ERR_INVALID_ARG, "a captured Adam step needs step_dev");
  *out = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_check(e, "hipStreamBeginCapture");
  gs_status st = gs_iteration_enqueue(it, stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(s, &graph);
  if (st != GS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_check(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_check(e, "hipGraphInstantiate");
  }
  gs_graph* gr = new gs_graph{graph, exec};
  *out = gr;
  return GS_OK;
}

gs_status gs_graph_launch(gs_graph* graph, void* stream) {
  if (!graph) return fail(GS_ERR_INVALID_ARG, "graph is null");
  return hip_check(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
}

gs_status gs_graph_time(gs_graph* graph, void* stream, int32_t warmup, int32_t reps,
                        float* ms_per_replay) {
  if (!graph || !ms_per_replay || warmup < 0 || reps < 1)
    return fail(GS_ERR_INVALID_ARG, "bad gs_graph_time arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int i = 0; e == hipSuccess && i < warmup; ++i) e = hipGraphLaunch(graph->exec, s);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int i = 0; e == hipSuccess && i < reps; ++i) e = hipGraphLaunch(graph->exec, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_check(e, "gs_graph_time");
  *ms_per_replay = ms / (float)reps;
  return GS_OK;
}

gs_status gs_graph_destroy(gs_graph* graph) {
  if (!graph) return GS_OK;
  hipError_t e1 = hipGraphExecDestroy(graph->exec);
  hipError_t e2 = hipGraphDestroy(graph->graph);
  delete graph;
  if (e1 != hipSuccess) return hip_check(e1, "hipGraphExecDestroy");
  return hip_check(e2, "hipGraphDestroy");
}

}  // extern "C"

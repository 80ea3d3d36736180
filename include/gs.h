/*
 * gs.h -- C ABI of the MI355X (gfx950) differentiable 3D Gaussian-splatting
 * rasterizer: the per-iteration hot path of the CaRtGS mapping back-end.
 *
 * The paper (CaRtGS, Sec. III-B) renders a keyframe from Gaussian primitives
 * with position p, quaternion q, scale s, opacity sigma and degree-3 SH
 * colour by alpha blending, Eq. (1), and refines the primitives by the loss
 * gradients of Eqs. (9)-(11) propagated back through the blend, Eqs. (2)-(4)
 * (Sec. III-C-1); the optimiser is that of 3DGS, which the paper retains
 * (Sec. IV-A).  One mapping iteration is
 *
 *     gs_preprocess -> gs_bin_sort -> gs_render_fwd -> gs_render_bwd
 *     (-> gs_adam_step)
 *
 * over one or more keyframes ("views").
 *
 * Conventions (all entry points):
 *   - Every function returns gs_status; GS_OK on success.  Argument checks
 *     are synchronous and happen before anything is enqueued; on error
 *     nothing is enqueued and gs_last_error() (thread-local) describes it.
 *   - Device-side conditions never fail a call.  They are reported through
 *     int32 flags inside the workspace (gs_flags_ptr): pair-capacity overflow
 *     and the count of Gaussians culled for non-finite parameters.  After an
 *     overflow, the downstream kernels of that iteration see zero pairs and
 *     their outputs are invalid; the Adam step of a whole iteration
 *     (gs_iteration_enqueue, graph replays) then changes no parameter, moment
 *     or step counter.  The caller re-plans with a larger capacity.
 *   - Ownership: every buffer is owned by the caller.  Calls never allocate
 *     device memory, never free it and never synchronise with the host.
 *     Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *     null stream) and is safe to capture with hipStreamBeginCapture.  The
 *     only library-owned objects are gs_graph handles (host objects holding
 *     an instantiated HIP graph), which the caller destroys.
 *   - Floating-point data are float32; image buffers are concatenated over
 *     views in view order: colour planar [3][H][W] per view, depth, T_final
 *     and last [H][W] per view.
 *   - Calls on distinct workspaces are independent and may run concurrently;
 *     calls that share a workspace must be stream-ordered.
 */
#ifndef GS_H_
#define GS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gs_status;
#define GS_OK 0
#define GS_ERR_INVALID_ARG 1  /* null/misaligned pointer, bad size, plan mismatch */
#define GS_ERR_UNSUPPORTED 2  /* sh_degree > 3, tile shape not 8x8/16x16/16x8, ... */
#define GS_ERR_HIP 3          /* a HIP runtime call or kernel launch failed */

#define GS_MAX_VIEWS 64
/* Device camera record, 20 float32 per view:
 *   fx fy cx cy | R[9] (world->camera rotation, row-major) | t[3] | near | bg[3]
 * x_cam = R x_world + t; image x right, y down, z forward; pixel (i, j)
 * is sampled at (i + 0.5, j + 0.5).  Image sizes come from the plan. */
#define GS_CAMERA_FLOATS 20

/* gs_raster_cfg.flags */
#define GS_CUTOFF_3SIGMA (1u << 0)    /* tile box from 3 sqrt(lambda_max) instead of the
                                         exact alpha >= 1/255 box (comparison only) */
#define GS_FUSED_L1 (1u << 1)         /* gs_render_bwd derives dL/dC, dL/dD from the L1
                                         loss against the targets instead of inputs */
#define GS_ACCUMULATE_GRADS (1u << 2) /* gs_render_bwd adds into the gradient buffers */
#define GS_PERSISTENT (1u << 3)       /* render kernels are resident and walk the
                                         tiles in chunks with a static stride (in
                                         either mode tiles with long lists run
                                         first, the order gs_bin_sort writes) */
#define GS_SPLAT_BWD (1u << 4)        /* splat-wise backward (Sec. III-C-1, Fig. 4a):
                                         the forward stores per-pixel (T, RGB, D) states
                                         at every 64th splat of a tile; the backward
                                         gives each lane one splat of a 64-splat bucket
                                         and streams pixel states across the lanes */
#define GS_RADIX_BIN (1u << 5)        /* gs_bin_sort by two stable radix sorts (the
                                         visible records by depth, then their pairs,
                                         generated in depth order, by tile id) instead
                                         of per-tile slot claims and per-tile sorts;
                                         the projection then counts no pairs per
                                         tile (the lists give the counts); same
                                         lists, bit for bit.  The raster kernels
                                         then read each pair's record through its
                                         record id (no copy of the records in list
                                         order).  About 20 B per record more and
                                         52 B per pair of capacity less workspace */

/* Gaussian parameters (Sec. III-B): SoA, float32, device pointers. */
typedef struct gs_gaussians {
  const float* means;          /* [n][3] world position p */
  const float* log_scales;     /* [n][3] s = exp(log_scales) */
  const float* quats;          /* [n][4] (w, x, y, z); normalised inside */
  const float* opacity_logits; /* [n]    opacity = sigmoid(logit) */
  const float* sh;             /* [n][(deg+1)^2][3] real SH coefficients */
  int64_t n;
  int32_t sh_degree;           /* 0..3 */
} gs_gaussians;

/* Gradients, same layout as gs_gaussians, device pointers (all required). */
typedef struct gs_gaussian_grads {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
} gs_gaussian_grads;

typedef struct gs_raster_cfg {
  int32_t tile_w;       /* 8 or 16 */
  int32_t tile_h;       /* 8 or 16 (16x16, 16x8, 8x8) */
  int32_t chunk;        /* tiles per work item in GS_PERSISTENT mode, 1..16 */
  int32_t lds_batch;    /* records staged in LDS per batch: 64, 128 or 256 */
  uint32_t flags;       /* GS_* flags above */
  float lambda_depth;   /* weight of the depth term of the fused L1 loss */
} gs_raster_cfg;

/* Execution plan: sizes, per-view tile/pixel offsets and the workspace
 * layout.  Caller-allocated, filled by gs_plan_init, read-only afterwards;
 * host memory, opaque. */
typedef struct gs_plan {
  uint64_t opaque[640];
} gs_plan;

/* Fill `plan` for n Gaussians of SH degree sh_degree rendered into n_views
 * views of sizes view_wh (host array [n_views][2] = width, height), with up
 * to pair_capacity (Gaussian, tile) pairs in total over all views.
 * Errors: GS_ERR_INVALID_ARG (n < 0, n_views not in 1..GS_MAX_VIEWS, a
 * width/height not in 1..16384, pair_capacity not in 1..2^31-1, more than
 * 2^31-1 records or pixels), GS_ERR_UNSUPPORTED (degree or tile shape). */
gs_status gs_plan_init(gs_plan* plan, int64_t n, int32_t sh_degree, int32_t n_views,
                       const int32_t* view_wh, const gs_raster_cfg* cfg,
                       int64_t pair_capacity);

/* Bytes of device workspace the plan needs (256-byte aligned base).  A new
 * workspace must be zero-filled once before its first use: a whole
 * iteration (gs_iteration_enqueue, graph replays) does not clear its
 * per-tile pair counters, relying on the binning of the previous iteration
 * or gs_bin_sort having left them zero.  gs_preprocess called on its own
 * clears them; calling it and then a whole iteration without gs_bin_sort in
 * between makes that iteration report a pair overflow (flag [0]). */
size_t gs_workspace_size(const gs_plan* plan);

/* Queries: total pixels over views, pixel offset of a view, total tiles. */
int64_t gs_plan_total_pixels(const gs_plan* plan);
int64_t gs_plan_pixel_offset(const gs_plan* plan, int32_t view);
int64_t gs_plan_total_tiles(const gs_plan* plan);

/* Device pointer to the int32 flags inside `ws`:
 *   [0] pair-capacity overflow (0/1)   [1] Gaussians culled as non-finite
 *       by the last gs_preprocess (published by the gs_bin_sort after it)
 *   [2] pair count P of the last gs_bin_sort (valid if [0] == 0)
 *   [3] visible (view, Gaussian) records (non-empty tile box) of the last
 *       gs_preprocess, counted by the gs_bin_sort after it
 *   [6] pairs the last gs_bin_sort needed (saturated at 2^31-1) */
int32_t* gs_flags_ptr(const gs_plan* plan, void* ws);

/* Byte offset inside the workspace of an intermediate array, for
 * inspection by tests and tools (-1 for an unknown region):
 *   GS_WS_RECORDS       [n_views*n] 64-byte records: f64 mean x, y;
 *                       f32 t, s1, s2, lo, depth, r, g, b, opacity;
 *                       u32 clamp bits, pad.  With the conic
 *                       Q = [[a,b],[b,c]] and d = mean - pixel, the
 *                       splat's opacity x Gaussian is 2^e with
 *                       e = lo - s1 (dx + t dy)^2 - s2 (dy - t dx)^2
 *                       = log2(opacity) - log2(e)/2 d^T Q d ((1, t): the
 *                       footprint axis nearer to x, |t| <= 1)
 *   GS_WS_RECTS         [n_views*n] u16 x0, y0, x1, y1 (tile box, exclusive)
 *   GS_WS_TILES_TOUCHED [n_views*n] u32
 *   GS_WS_PAIR_OFFSETS  [n_views*n] u32, first pair of each visible record
 *   GS_WS_SORTED_KEYS   [P] u64 after gs_bin_sort: global tile id << 32 |
 *                       float32 bits of depth
 *   GS_WS_SORTED_VALS   [P] u32 (pair index in generation order)
 *   GS_WS_SORTED_RECS   [P] u32 (record index v*n + i of each sorted pair)
 *   GS_WS_RANGES        [total_tiles][2] u32 [start, end) of each tile's
 *                       list, (0, 0) for a tile without pairs */
#define GS_WS_RECORDS 0
#define GS_WS_RECTS 1
#define GS_WS_TILES_TOUCHED 2
#define GS_WS_PAIR_OFFSETS 3
#define GS_WS_SORTED_KEYS 4
#define GS_WS_SORTED_VALS 5
#define GS_WS_SORTED_RECS 6
#define GS_WS_RANGES 7
int64_t gs_plan_ws_offset(const gs_plan* plan, int32_t region);

/* a1. Per (view, Gaussian): activations, quaternion rotation, 3D covariance,
 * camera transform, near cull (z <= near), EWA 2D covariance with 0.3 px^2
 * dilation and Jacobian clamped at 1.3x the half FOV, conic, exact tile box
 * of the alpha >= 1/255 ellipse, SH colour clamped at 0, depth.  Gaussians
 * with non-finite parameters or a zero quaternion are culled and counted.
 * (Sec. III-B: parameters p, q, s, sigma, SH; alpha from a projected 2D
 * Gaussian times opacity.)  cams_dev: device [n_views][GS_CAMERA_FLOATS].
 * g->n and g->sh_degree must equal the plan's. */
gs_status gs_preprocess(const gs_plan* plan, const gs_gaussians* g, const float* cams_dev,
                        void* ws, void* stream);

/* a2. Tile binning (the per-tile depth-sorted lists of Sec. III-C-1).
 * Pairs are the (record, tile) incidences of the tile boxes, numbered in
 * generation order (record-major, row-major tiles).  Each tile's list is
 * ordered by (float32 depth, generation index): ties in depth keep Gaussian
 * order, so the lists are unique and bit-exact.  Needs the per-tile and
 * per-chunk (64 Gaussians of a view) pair counts of the gs_preprocess call
 * just before on the same workspace.  Also writes the render kernels' work
 * order: tiles with at least 32 pairs first, in tile order, then the others
 * in reverse tile order (results do not depend on the order).
 * Overflow of the plan's pair capacity sets flag [0]. */
gs_status gs_bin_sort(const gs_plan* plan, void* ws, void* stream);

/* a3. Front-to-back compositing of Eq. (1) per pixel over its tile's sorted
 * list: alpha = min(0.99, o G); skip if the exponent is positive or alpha <
 * 1/255; stop before blending when T (1 - alpha) < 1e-4.  Outputs (device,
 * concatenated over views): color [3][H][W] = sum c alpha T + T_final bg,
 * depth [H][W] = sum z alpha T (camera z, unnormalised), T_final [H][W],
 * last [H][W] = 1 + position in the tile list of the last blended Gaussian
 * (0 if none).  If target_rgb is non-null, loss_per_view[v] receives the L1
 * loss mean|C - C*| + lambda_depth mean|D - D*| (depth term only if
 * target_depth is non-null); loss_per_view may be null otherwise.  cams_dev
 * supplies the background colour of each view. */
gs_status gs_render_fwd(const gs_plan* plan, void* ws, const float* cams_dev, float* color,
                        float* depth, float* T_final, uint32_t* last, const float* target_rgb,
                        const float* target_depth, float* loss_per_view, void* stream);

/* a4-a6. Backward of one iteration (Eqs. (2)-(4)).  Default (pixel-wise):
 * per pixel, back to front from its last blended Gaussian, with the
 * transmittance recomputed by division from T_final; per-pair gradients are
 * reduced across the tile's wavefront.  With GS_SPLAT_BWD (splat-wise,
 * Sec. III-C-1): one lane per splat of a 64-splat bucket, pixel states
 * resumed from those the forward stored and handed from lane to lane.
 * Either way the per-pair gradients are then summed per Gaussian in a fixed
 * order (deterministic) and carried through the projection to the
 * parameters.  Upstream gradients
 * are dL_dcolor [3][H][W] and dL_ddepth [H][W] (nullable: zero), or, with
 * GS_FUSED_L1, those of the L1 loss of gs_render_fwd against target_rgb and
 * target_depth (sign(0) = 0).  `out` is overwritten (GS_ACCUMULATE_GRADS:
 * added to).  dL_dpose (nullable) receives [n_views][6] = (rho, phi), the
 * gradient w.r.t. a left perturbation R <- Exp(phi) R, t <- Exp(phi) t + rho
 * of each view's pose at zero (overwritten).  The forward buffers must be
 * those written by gs_render_fwd with the same plan and workspace. */
gs_status gs_render_bwd(const gs_plan* plan, const gs_gaussians* g, const float* cams_dev,
                        void* ws, const float* color, const float* depth,
                        const float* T_final, const uint32_t* last,
                        const float* dL_dcolor, const float* dL_ddepth,
                        const float* target_rgb, const float* target_depth,
                        const gs_gaussian_grads* out, float* dL_dpose, void* stream);

/* a4, full Eq. (9).  Rendered loss and its image gradients, per view:
 *   L_v = (1 - lambda_ssim) mean|C - C*| + lambda_ssim (1 - SSIM(C, C*))
 *         + lambda_depth mean|D - D*|          (lambda_depth from the plan)
 * with the SSIM of 3DGS (per channel, 11x11 Gaussian window of sigma 1.5,
 * zero padding, C1 = 0.01^2, C2 = 0.03^2, mean over pixels and channels;
 * sign(0) = 0 in the L1 terms).  Writes dL_dcolor [3][H][W] and dL_ddepth
 * [H][W] (device, concatenated over views) -- the explicit upstream
 * gradients of gs_render_bwd -- and loss_per_view (nullable).
 * target_depth is nullable (no depth term). */
gs_status gs_render_loss(const gs_plan* plan, void* ws, const float* color, const float* depth,
                         const float* target_rgb, const float* target_depth, double lambda_ssim,
                         float* dL_dcolor, float* dL_ddepth, float* loss_per_view, void* stream);

/* The two stages of gs_render_bwd as separate calls (same arguments, same
 * checks).  a5: gs_render_bwd_raster runs the per-pixel backward and leaves
 * one 10-float partial gradient (rgb, depth, opacity, conic a b c, mean x y)
 * per (tile, Gaussian) pair in the workspace.  a6: gs_project_bwd reduces
 * those partials per Gaussian in a fixed order and applies the chain rule to
 * the parameters and the camera tangents. */
gs_status gs_render_bwd_raster(const gs_plan* plan, void* ws, const float* cams_dev,
                               const float* color, const float* depth, const float* T_final,
                               const uint32_t* last, const float* dL_dcolor,
                               const float* dL_ddepth, const float* target_rgb,
                               const float* target_depth, void* stream);
gs_status gs_project_bwd(const gs_plan* plan, const gs_gaussians* g, const float* cams_dev,
                         void* ws, const gs_gaussian_grads* out, float* dL_dpose, void* stream);

/* a7. One Adam step over several parameter groups in a single launch
 * (torch.optim.Adam semantics without weight decay, the 3DGS optimiser):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
 * Groups are a host array of device pointers.  If a group has
 * opacity_reg != 0, the gradient of lambda_o * mean_i |sigmoid(p_i)| over
 * reg_count Gaussians (Eq. (10)) is added to g first (p is a logit).
 * Hyper-parameters are doubles: 1 - beta and the bias corrections are formed
 * in double precision and rounded once, as torch does for float32 params.
 * step_dev (nullable): device int32 step counter; when given, t = *step_dev
 * + 1 is read on the device and written back after the update (for graph
 * replays), and `step` is ignored.  Pointers must be 16-byte aligned. */
typedef struct gs_param_group {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr;
  int32_t opacity_reg;
} gs_param_group;

gs_status gs_adam_step(const gs_param_group* groups, int32_t n_groups, int32_t step,
                       double beta1, double beta2, double eps, double lambda_o,
                       int64_t reg_count, int32_t* step_dev, void* stream);

/* Camera-pose tangent of the autograd path (the camera gradient of the
 * render, Sec. III-B; the mapping back-end refines keyframe poses with the
 * map).  gs_render_bwd's dL_dpose is the gradient w.r.t. a left perturbation
 * delta = (rho, phi) of each view's world->camera pose at zero.  A caller
 * that optimises a tangent xi renders with the retracted pose and pulls the
 * gradient back to xi:
 *
 * gs_pose_retract: for each view v, cams_out[v] = cams_in[v] with
 *   R' = Exp(phi) R,  t' = Exp(phi) t + rho      (xi[v] = (rho, phi))
 * Exp is the SO(3) exponential (Rodrigues); computed in FP64 from the
 * float32 inputs and rounded once to float32; the other record fields are
 * copied.  cams_in, cams_out: device [n_views][GS_CAMERA_FLOATS] (may be the
 * same buffer); xi: device float [n_views][6].
 *
 * gs_pose_tangent_vjp: given dL_ddelta [n_views][6] at the retracted pose,
 * writes dL_dxi [n_views][6]:
 *   dL/drho = g_rho,   dL/dphi = J(phi)^T (g_phi - rho x g_rho)
 * with J the left Jacobian of SO(3) (Exp(phi + dphi) = Exp(J dphi) Exp(phi)
 * to first order).  At xi = 0 it is the identity.  Device buffers; dL_dxi
 * may alias dL_ddelta.
 * Errors: GS_ERR_INVALID_ARG (null pointer, n_views not in 1..GS_MAX_VIEWS). */
gs_status gs_pose_retract(const float* cams_in, const float* xi, float* cams_out,
                          int32_t n_views, void* stream);
gs_status gs_pose_tangent_vjp(const float* xi, const float* dL_ddelta, float* dL_dxi,
                              int32_t n_views, void* stream);

/* Adaptive densification and opacity pruning (Sec. IV-A: densify every 500
 * iterations with a positional-gradient threshold tau_p, remove Gaussians
 * with opacity below eps_alpha; clone and split as in 3DGS).
 *
 * gs_grad_stats, after gs_render_bwd(_raster) of an iteration: for every
 * Gaussian visible in a view, accum[i] += |(g_x W/2, g_y H/2)| (the 2D mean
 * gradient in normalised device coordinates) and denom[i] += 1.
 * accum, denom: device float[n], caller-owned, zeroed by the caller at the
 * start of a densification interval.
 *
 * gs_densify_prune: Gaussian i is selected when denom > 0 and accum/denom >=
 * tau_p; a selected Gaussian is cloned (itself + a copy) when its largest
 * scale is <= percent_dense * extent, otherwise split into two children with
 * means p + R(q)(s * n_k), n_k = normals[i][k][0..2] (caller's standard
 * normal draws, device float[n][2][3]) and scales s / 1.6.  Every output
 * Gaussian with sigmoid(logit) < eps_alpha is dropped.  Output order is the
 * input order (a copy right after its original, two children in place of
 * their parent); Adam moments `m`, `v` are carried for kept originals and
 * zero for copies and children.  Decisions are taken in FP32.  The output
 * count is written to *n_out (device int32); at most out_capacity Gaussians
 * are written (the caller compares *n_out with its capacity).  tmp: device
 * scratch of gs_densify_tmp_bytes(n) bytes, 256-byte aligned. */
gs_status gs_grad_stats(const gs_plan* plan, void* ws, float* accum, float* denom, void* stream);
size_t gs_densify_tmp_bytes(int64_t n);
gs_status gs_densify_prune(const gs_gaussians* g, const gs_gaussian_grads* m,
                           const gs_gaussian_grads* v, const float* accum, const float* denom,
                           const float* normals, float tau_p, float eps_alpha,
                           float percent_dense, float extent, const gs_gaussian_grads* out,
                           const gs_gaussian_grads* out_m, const gs_gaussian_grads* out_v,
                           int64_t out_capacity, int32_t* n_out, void* tmp, void* stream);

/* Stand-alone stable LSD radix sort of n (key, value) pairs on the low
 * key_bits bits of the keys (1..64).
 * keys/vals are device arrays, sorted in place; tmp is device scratch of
 * gs_sort_tmp_bytes(n) bytes. */
size_t gs_sort_tmp_bytes(int64_t n);
gs_status gs_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits,
                        void* tmp, void* stream);

/* Allocation-free form of gs_sort_pairs, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, hosts that
 * forbid hipMalloc).  Same arguments and result as gs_sort_pairs without
 * tmp: the scratch is a device array inside the library, one per GPU, of
 * GS_SORT_NOALLOC_MAX pairs (about 12.9 MB), held from the first call on
 * that GPU until the process ends.  n above GS_SORT_NOALLOC_MAX is
 * rejected with GS_ERR_INVALID_ARG before any GPU work.  No hipMalloc,
 * hipFree or allocating library routine is called.  Every call on one GPU
 * shares that GPU's scratch: calls that overlap in time on one GPU (two
 * streams, two host threads) race and must be ordered by the caller. */
#define GS_SORT_NOALLOC_MAX (1 << 20)
gs_status gs_sort_pairs_noalloc(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits,
                                void* stream);

/* Spatial layout of a Gaussian pool (a data-layout step between iterations,
 * e.g. when the mapping loop re-plans after densification, Sec. IV-A).
 * gs_spatial_order writes the permutation perm [n] (device int32) that
 * sorts the means [n][3] by their Morton code in the pool's bounding box
 * (10 bits per axis; ties keep the index order; a NaN mean goes last);
 * tmp is device scratch of gs_spatial_order_tmp_bytes(n) bytes, 256-byte
 * aligned.  gs_permute_gaussians writes dst[j] = src[perm[j]] for the five
 * parameter arrays (use it for the Adam moments too; dst must not alias
 * src).  Rendering a permuted pool gives the same images up to the order
 * of exact depth ties. */
size_t gs_spatial_order_tmp_bytes(int64_t n);
gs_status gs_spatial_order(const float* means, int64_t n, int32_t* perm, void* tmp, void* stream);
gs_status gs_permute_gaussians(const gs_gaussians* src, const int32_t* perm,
                               const gs_gaussian_grads* dst, void* stream);

/* a8. Whole-iteration hipGraph.  The mapping back-end re-optimises keyframes
 * of a growing pool again and again (Sec. III-C-2, Eqs. (5)-(8)); the paper
 * takes one keyframe per iteration, this form takes a batch of keyframes of
 * any resolutions over one shared Gaussian pool per iteration.  The
 * descriptor names every buffer of one mapping iteration; gs_graph_create
 * captures gs_preprocess, gs_bin_sort, gs_render_fwd, gs_render_bwd and (if
 * n_adam_groups > 0) gs_adam_step on `stream` and instantiates the graph.
 * Poses, parameters and targets live in device memory, so replays see their
 * current values.  An iteration with Adam needs step_dev (the device step
 * counter, advanced once per iteration unless the pairs overflow);
 * gs_iteration_enqueue and gs_graph_create reject a null one.
 * With one view, Adam groups and no GS_ACCUMULATE_GRADS, the gradient
 * buffers are written for the Gaussians that have pairs only: Adam takes the
 * others' gradients as zero, so their entries in `grads` are left as they
 * were (the parameters and moments are those of a fully written gradient). */
/* Keyframe pool of a scheduled batch (gs_iteration.gather,
 * gs_gather_views): every keyframe has the resolution of every view of the
 * plan.  Device pointers: pool_cams [n_pool][GS_CAMERA_FLOATS], pool_rgb
 * [n_pool][3][H][W], pool_depth [n_pool][H][W] (nullable: no depth target),
 * sel [n_views] keyframe ids (an id outside [0, n_pool) leaves its slot as
 * it was). */
typedef struct gs_view_gather {
  const float* pool_cams;
  const float* pool_rgb;
  const float* pool_depth;
  const int32_t* sel;
  int32_t n_pool;
} gs_view_gather;

/* Copies the selected keyframes into the batch slots (the first launch of an
 * iteration with `gather`): cams_out [n_views][GS_CAMERA_FLOATS], rgb_out
 * [n_views][3][H][W], depth_out [n_views][H][W] (null iff pool_depth is).
 * Errors: GS_ERR_INVALID_ARG (null pointer, n_pool < 1, views of differing
 * sizes). */
gs_status gs_gather_views(const gs_plan* plan, const gs_view_gather* g, float* cams_out,
                          float* rgb_out, float* depth_out, void* stream);

typedef struct gs_iteration {
  const gs_plan* plan;
  void* ws;
  gs_gaussians gaussians;
  const float* cams_dev;
  float* color;
  float* depth;
  float* T_final;
  uint32_t* last;
  const float* target_rgb;
  const float* target_depth;
  float* loss_per_view;
  const float* dL_dcolor;
  const float* dL_ddepth;
  gs_gaussian_grads grads;
  float* dL_dpose;
  const gs_param_group* adam_groups; /* host array, copied at creation */
  int32_t n_adam_groups;
  int32_t* step_dev;
  double beta1, beta2, eps, lambda_o;
  int64_t reg_count;
  /* lambda_ssim > 0: the loss of gs_render_loss (Eq. (9) with SSIM) is
   * evaluated after the forward into loss_per_view, its image gradients into
   * loss_grad_color / loss_grad_depth, which then drive the backward (the
   * plan must not set GS_FUSED_L1).  0: fused L1 or explicit dL_dcolor. */
  double lambda_ssim;
  float* loss_grad_color;
  float* loss_grad_depth;
  /* Optional (null: off): the batch's views are keyframes of a pool, chosen
   * per iteration by the keyframe scheduler (Sec. III-C-2, Eqs. (5)-(8)).
   * The iteration first copies, for every batch slot b, keyframe sel[b]'s
   * camera record into cams_dev[b] and its target images into target_rgb /
   * target_depth slot b (those buffers are overwritten), so a captured graph
   * renders whatever ids the caller last wrote to sel -- no re-capture. */
  const struct gs_view_gather* gather;
} gs_iteration;

typedef struct gs_graph gs_graph;

gs_status gs_iteration_enqueue(const gs_iteration* it, void* stream);
gs_status gs_graph_create(const gs_iteration* it, void* stream, gs_graph** out);
gs_status gs_graph_launch(gs_graph* graph, void* stream);
gs_status gs_graph_destroy(gs_graph* graph);

/* Autotuner timing core: replays `graph` warmup + reps times on `stream`
 * and returns the mean milliseconds per replay of the timed reps, measured
 * with HIP events on that stream.  Synchronises the stream (a measurement
 * call, not for the iteration loop). */
gs_status gs_graph_time(gs_graph* graph, void* stream, int32_t warmup, int32_t reps,
                        float* ms_per_replay);

/* Per-launch timing of one eagerly enqueued iteration (measurement call, not
 * for the iteration loop, never under capture).  Enqueues `warmup`
 * iterations of `it`, then `reps` iterations with a HIP event recorded on
 * `stream` at each mark below, synchronises, and writes the milliseconds
 * between consecutive marks: ms[r * (GS_N_MARKS - 1) + k] is the span from
 * mark k to mark k + 1 of rep r (host array of reps * (GS_N_MARKS - 1)).
 * A span whose launches the iteration does not make (no SSIM term, short
 * lists sorted by the forward) is the empty span between two marks. */
#define GS_MARK_START 0
#define GS_MARK_PREPROCESS 1       /* after the counter clear and the projection */
#define GS_MARK_BIN_SCAN 2         /* after the binning's scans */
#define GS_MARK_BIN_SCATTER 3      /* after the pair scatter (GS_RADIX_BIN: after the
                                      depth sort of the records and the pair
                                      generation) */
#define GS_MARK_BIN_SHORT_SORT 4   /* after the per-tile sorts of short lists
                                      (GS_RADIX_BIN: after the tile-id passes) */
#define GS_MARK_BIN_LONG_SORT 5    /* after the long-list sorts (GS_RADIX_BIN: after
                                      the per-tile counts, their scan and the
                                      per-tile pass) */
#define GS_MARK_FORWARD 6          /* after compositing (and the L1 loss sums) */
#define GS_MARK_LOSS 7             /* after the SSIM loss kernels */
#define GS_MARK_RASTER_BWD 8       /* after the raster backward */
#define GS_MARK_PROJECT_BWD 9      /* after the projection backward */
#define GS_MARK_ADAM 10            /* after Adam and its step advance */
#define GS_N_MARKS 11
gs_status gs_iteration_time_marks(const gs_iteration* it, void* stream, int32_t warmup,
                                  int32_t reps, float* ms);

/* Adaptive keyframe selection, host only (Sec. III-C-2, Eqs. (5)-(8)).
 * A keyframe enters the pool with r0 remaining optimisations and loss +inf;
 * gs_sched_select draws `batch` distinct keyframes uniformly among those
 * with r > 0 -- uniforms[b] in [0, 1) picks position floor(u m) of the m
 * eligible keyframes in index order -- and decrements their counts; when no
 * keyframe is eligible it first resets every count by Eq. (8): 2 for the
 * d_k = max(1, floor(k / d)) largest reported losses (ties to the lower
 * index), 1 otherwise.  gs_sched_report stores a keyframe's latest loss.
 * All storage is the caller's (r: int32[capacity], l: double[capacity]).
 * batch = 1 is the paper's one-keyframe-per-iteration rule. */
typedef struct gs_scheduler {
  int32_t* r;
  double* l;
  int32_t capacity;
  int32_t count;
  int32_t r0;
  int32_t d;
  int64_t refills;
} gs_scheduler;

gs_status gs_sched_init(gs_scheduler* s, int32_t* r, double* l, int32_t capacity, int32_t r0,
                        int32_t d);
gs_status gs_sched_add_keyframe(gs_scheduler* s, int32_t* out_id);
gs_status gs_sched_select(gs_scheduler* s, int32_t batch, const double* uniforms,
                          int32_t* out_ids, int32_t* out_count);
gs_status gs_sched_report(gs_scheduler* s, int32_t id, double loss);
const char* gs_sched_last_error(void);

const char* gs_status_string(gs_status s);
const char* gs_last_error(void);
int32_t gs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H_ */

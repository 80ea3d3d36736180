// Internal definitions of the gfx950 rasterizer library: the plan stored in
// gs_plan's opaque words, the 64-byte projected record, the per-view tables
// passed to kernels by value, and wave64 helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/gs.h"

namespace gs {

constexpr int kWave = 64;
constexpr int kMaxViews = GS_MAX_VIEWS;
constexpr uint32_t kPlanMagic = 0x67735031u;  // "gsP1"

// Flags in the workspace (int32).  See gs_flags_ptr.
enum Flag : int {
  F_OVERFLOW = 0,
  F_NONFINITE = 1,
  F_PAIRS = 2,
  F_VISIBLE = 3,
  F_QUEUE_FWD = 4,
  F_QUEUE_BWD = 5,
  F_PAIRS_WANTED = 6,
  F_LONG_TILES = 7,  // tiles whose lists go to the long-list sort
  F_BQ_FULL = 8,     // splat-wise buckets with more than 32 pairs
  F_BQ_HALF = 9,     // splat-wise buckets with at most 32 pairs
  F_NF_ACC = 10,     // non-finite Gaussians counted by the projection, published
                     // in F_NONFINITE (and cleared) by the binning scan
  F_COUNT = 16
};

// Per-view geometry of the tile grid and of the concatenated image buffers.
struct ViewInfo {
  int32_t W, H;
  int32_t tiles_x, tiles_y;
  int32_t tile_off;  // first global tile id of this view
  int32_t pix_off;   // first pixel of this view in the concatenated buffers
};

struct ViewTable {
  int32_t n_views;
  int32_t total_tiles;
  int32_t tw, th;
  int64_t total_pix;
  ViewInfo v[kMaxViews];
};

// Projected (view, Gaussian) record, 64 bytes.  The splat's base-2
// exponent at offset d = (dx, dy) = mean - sample point is kept in the
// eigen form of its conic Q = [[a, b], [b, c]]:
//   log2(o) - log2(e)/2 d^T Q d = lo - s1 (dx + t dy)^2 - s2 (dy - t dx)^2
// (1, t) is the footprint axis nearer to x (|t| <= 1), (-t, 1) the other,
// s1, s2 the eigenvalues times log2(e)/2 / (1 + t^2), lo = log2(o).  The
// offset is formed in FP64 (no cancellation at large pixel coordinates),
// the rest in FP32 as a sum of squares (no cancellation for elongated
// footprints).  The forward reads the first 48 bytes of a record per splat.
struct __align__(16) Rec {
  double mx, my;     // 2D mean, pixels
  float t, s1, s2;   // first axis slope; exponent scales along (1, t), (-t, 1)
  float lo;          // log2(opacity)
  float z;           // camera-space depth
  float r, g, b;     // colour after the clamp at 0
  float o;           // opacity
  uint32_t clamp;    // bit ch set: channel ch was clamped at 0 (no gradient)
  uint32_t pad[2];
};
static_assert(sizeof(Rec) == 64, "record must be 64 bytes");
constexpr double kLog2e = 1.4426950408889634;  // log2(e)
constexpr double kLn2 = 0.6931471805599453;    // ln(2), its inverse

// Base-2 exponent of record r at offset (dx, dy) = mean - sample point (the
// FP64 difference rounded to FP32): the splat's opacity times its Gaussian
// is 2^that.  Never above lo <= 0.
__device__ __forceinline__ float rec_exponent(const Rec& r, float dx, float dy) {
  const float p = fmaf(r.t, dy, dx), q = fmaf(-r.t, dx, dy);
  const float u = r.s1 * p, w = r.s2 * q;
  return fmaf(-u, p, fmaf(-w, q, r.lo));
}

// The conic [[a, b], [b, c]] of record r (natural exponent -d^T Q d / 2),
// for the mean gradient.
__device__ __forceinline__ void rec_conic(const Rec& r, float& a, float& b, float& c) {
  const float sc = (float)(2.0 * kLn2), tt = r.t * r.t;  // 1 / (log2(e) / 2)
  a = sc * fmaf(r.s2, tt, r.s1);
  b = sc * (r.t * (r.s1 - r.s2));
  c = sc * fmaf(r.s1, tt, r.s2);
}

// Where the raster kernels read the records of the tile lists: a copy in
// list order written by the binning (idx null: list position k is base[k]),
// or the per-view record array itself, through each pair's record id
// (base[idx[k]]).
struct RecSrc {
  const Rec* base;
  const uint32_t* idx;
  __device__ __forceinline__ const Rec* at(uint32_t k) const {
    return idx ? base + idx[k] : base + k;
  }
};

// Per-pair gradient partial written by the backward raster kernel:
// rgb(3), depth, opacity, conic a b c, mean x y: ten floats, 40 bytes, so
// slots are 8-byte aligned and move as five float2.
constexpr int kPairGrad = 10;
struct PairSlot {
  float4 a, b;  // rgb, depth | opacity, conic a b c
  float2 c;     // mean x y
};
__device__ __forceinline__ PairSlot load_pair(const float* gp, int64_t k) {
  const float2* p = reinterpret_cast<const float2*>(gp + k * kPairGrad);
  const float2 p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3], p4 = p[4];
  return PairSlot{make_float4(p0.x, p0.y, p1.x, p1.y), make_float4(p2.x, p2.y, p3.x, p3.y), p4};
}
// the colour partials alone (the first two float2)
__device__ __forceinline__ float4 load_pair_colour(const float* gp, int64_t k) {
  const float2* p = reinterpret_cast<const float2*>(gp + k * kPairGrad);
  const float2 p0 = p[0], p1 = p[1];
  return make_float4(p0.x, p0.y, p1.x, p1.y);
}
__device__ __forceinline__ void store_pair(float* gp, int64_t k, float4 a, float4 b, float2 c) {
  float2* p = reinterpret_cast<float2*>(gp + k * kPairGrad);
  p[0] = make_float2(a.x, a.y);
  p[1] = make_float2(a.z, a.w);
  p[2] = make_float2(b.x, b.y);
  p[3] = make_float2(b.z, b.w);
  p[4] = c;
}

struct Plan {
  uint32_t magic;
  int32_t deg, K, n_views;
  int64_t n;        // Gaussians
  int64_t n_rec;    // n_views * n
  int64_t pair_cap;
  gs_raster_cfg cfg;
  int32_t tile_bits, pad0;
  int64_t chunks_per_view;   // chunks of 64 Gaussians per view (one wavefront each)
  int64_t n_chunks;          // n_views * chunks_per_view
  int64_t proj_blocks;       // blocks of the projection backward
  ViewTable vt;
  // workspace layout (byte offsets from the 256-aligned base)
  size_t off_flags, off_rec, off_rect, off_tt, off_poff;
  size_t off_chunk_cnt, off_chunk_pre;  // per chunk: (pairs, visible) counts and offsets
  size_t off_vis_list;                  // visible records in index order
  size_t off_vis_clamp;                 // their colour clamp bits, same order
  size_t off_tile_cnt, off_tile_start, off_long;
  size_t off_keys, off_scatter, off_vals, off_pair_rec, off_sorted_rec, off_srec;
  size_t off_ranges, off_tile_last, off_tile_loss;
  size_t off_grad_pair, off_pose_part, off_order;
  // several views: per record, its projection-backward terms; per
  // Gaussian, the projection half's mean gradient
  size_t off_rec_terms, off_gp_tmp;
  size_t off_ssim_maps, off_ssim_part;
  // splat-wise backward: bucket offsets, bucket queues and their per-tile
  // positions, pixel states
  size_t off_boff, off_bq, off_ckpt, off_full_start, off_half_start;
  int64_t ckpt_slots;
  // binning scan: rounds (one block each when more than one) and their
  // per-channel partial sums
  int64_t scan_rounds;
  size_t off_scan_part;
  // radix binning (GS_RADIX_BIN): depth keys and record ids of the visible
  // records (two buffers each), tile keys, generation indices and record
  // ids of the pairs (two each), per-block digit counts, digit totals, and
  // the pair offsets of blocks of depth-sorted records
  size_t off_rb_dkey[2], off_rb_rid[2], off_rb_tkey[2], off_rb_gidx[2], off_rb_ridx[2];
  size_t off_rb_hist, off_rb_dtot, off_rb_part, off_rb_pay, off_rb_spay, off_rb_zrec;
  int64_t rb_rec_blocks, rb_pair_blocks;
  size_t ws_size;
};
static_assert(sizeof(Plan) <= sizeof(gs_plan), "plan does not fit gs_plan");

inline const Plan* plan_of(const gs_plan* p) { return reinterpret_cast<const Plan*>(p->opaque); }
inline Plan* plan_of(gs_plan* p) { return reinterpret_cast<Plan*>(p->opaque); }

template <typename T>
inline T* ws_at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// Radix sort geometry: 256 threads x 16 keys per block, 8-bit digits.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

constexpr int kProjThreads = 128;

// Splat-wise backward: splats per bucket (one per lane) and the floats of a
// stored pixel state (T, r, g, b, depth).
constexpr int kBucket = 64;
constexpr int kStateFloats = 5;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return (l == 0) ? 0ull : (~0ull >> (64 - l));
}

// (the builtin on the bool itself: HIP's __ballot takes an int, whose round
// trip through a VGPR costs two VALU per vote)
__device__ __forceinline__ uint64_t ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Orders a wavefront's LDS writes before its own later LDS reads (the lanes
// of one wavefront, no block barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave64 sum with the result valid in every lane: butterfly over xor
// distances 1..32.  Lanes that are inactive must hold 0.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_xor(x, o, kWave);
    x = x > y ? x : y;
  }
  return x;
}

// L1 loss of one view from its per-tile partials (float2: colour sum, depth
// sum): mean|C - C*| + lambda_depth mean|D - D*|.  The summation order is
// that of 1024 threads (thread t sums tiles t, t + 1024, ... in FP64; wave
// butterflies; the 16 wave sums in order), whatever the block size NT (a
// multiple of 64 dividing 1024), so every caller gets the same bits.  Every
// thread of the block must call; thread 0 writes *loss.
constexpr int kLossVirtual = 1024;
template <int NT>
__device__ __forceinline__ void loss_reduce_view(const float2* __restrict__ tl, int nt, double npx,
                                                 float lambda_depth, int has_depth,
                                                 float* __restrict__ loss) {
  static_assert(NT % kWave == 0 && kLossVirtual % NT == 0, "block size");
  constexpr int J = kLossVirtual / NT, VW = kLossVirtual / kWave;
  __shared__ double sa[VW], sb[VW];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int vt = j * NT + (int)threadIdx.x;  // virtual thread
    double a = 0.0, b = 0.0;
    for (int k = vt; k < nt; k += kLossVirtual) {
      const float2 x = tl[k];
      a += x.x;
      b += x.y;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane_id() == 0) {
      sa[vt / kWave] = a;
      sb[vt / kWave] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int k = 0; k < VW; ++k) {
      ta += sa[k];
      tb += sb[k];
    }
    *loss = (float)(ta / (3.0 * npx) + (has_depth ? lambda_depth * tb / npx : 0.0));
  }
}

// Step-dependent Adam factors of an iteration, computed once by its first
// launch (which also advances the device step counter): the bias
// corrections 1 - beta^t, 1/sqrt(1 - beta2^t) and lr_g / (1 - beta1^t) per
// parameter group, with the formulas the Adam kernel uses otherwise, so the
// values are the same bits.  Lives in the workspace's flag block.
constexpr int kAdamFoldGroups = 16;
struct AdamStepFactors {
  double bc1, bc2;
  float inv_bc2s;
  int32_t step;
  float step_size[kAdamFoldGroups];
};
// Timing marks of an eagerly enqueued iteration: event `k` (a GS_MARK_*
// index) is recorded on the launch stream after the launches before it.
struct Marks {
  hipEvent_t* ev = nullptr;  // GS_N_MARKS events, or null (no marks)
  hipError_t at(int k, hipStream_t s) const {
    return ev ? hipEventRecord(ev[k], s) : hipSuccess;
  }
};
struct StepAdvance {
  int32_t* step;
  double beta1, beta2;
  AdamStepFactors* out;
  int32_t n_groups;
  float lr[kAdamFoldGroups];
};
// One thread: advances the step counter and stores the factors of the new
// step t.
__device__ inline void advance_step(const StepAdvance& st) {
  const int32_t t = *st.step + 1;
  *st.step = t;
  AdamStepFactors* f = st.out;
  const double bc1 = 1.0 - pow(st.beta1, (double)t);
  const double bc2 = 1.0 - pow(st.beta2, (double)t);
  f->bc1 = bc1;
  f->bc2 = bc2;
  f->inv_bc2s = (float)(1.0 / sqrt(bc2));
  f->step = t;
  for (int g = 0; g < st.n_groups; ++g) f->step_size[g] = (float)((double)st.lr[g] / bc1);
}
constexpr size_t kBiasOffset = 128;  // bytes from the flags (F_COUNT int32 before it)
static_assert(kBiasOffset >= F_COUNT * 4 && kBiasOffset + sizeof(AdamStepFactors) <= F_COUNT * 16,
              "flag block");

// Work of a whole iteration that rides on the Adam launch: the step counter
// advanced at the iteration's start (Adam then reads the factors stored
// then), and the reduction of a one-view forward's per-tile L1 partials into
// *loss.
struct AdamFold {
  bool step_taken;
  const AdamStepFactors* factors;
  const float2* tile_loss;
  int32_t loss_tiles, loss_has_depth;
  double loss_pixels;
  float lambda_depth;
  float* loss;
};

// Host-side launch helpers (defined in the .hip files).
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);

}  // namespace gs

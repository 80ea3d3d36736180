// a3-a5: per-tile compositing (Eq. (1)), its pixel-wise backward
// (Eqs. (2)-(4)) and the splat-wise backward (Sec. III-C-1, below).  One wave64 per tile: a lane owns PPL = tile pixels / 64
// pixels (2x2 quads on 16x16 tiles, horizontal pairs on 16x8, one pixel on
// 8x8), so the per-Gaussian work that does not depend on the pixel -- the
// LDS read of the record, the wavefront reduction of the backward -- is
// shared by up to 256 pixels.  Single-wave workgroups need no workgroup
// barriers beyond LDS reuse, and many of them fit a CU.
//
// Forward: records of the tile's depth-sorted list are staged in LDS in
// batches; every lane walks the batch front to back for each of its pixels.
// The wavefront leaves as soon as the ballot of lanes with an unfinished
// pixel is empty.
//
// Backward: back to front from the tile's last used position.  Each lane
// recomputes alpha with the forward's code (so every skip decision is the
// forward's), undoes the transmittance by division from T_final and keeps
// the sums of what lies behind.  The ten per-pair partial gradients of a
// Gaussian are summed over the lane's pixels, then over the wavefront with
// DPP (skipped when no lane contributes), and written to the pair's own
// slot: no atomics, deterministic.
#include "tilesort.h"

namespace gs {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;

// alpha of record r at sample point (sx, sy): oG = opacity x Gaussian, a =
// oG clamped at 0.99.  Returns false when the Gaussian is skipped (alpha
// below 1/255; its exponent is never positive).
__device__ __forceinline__ bool eval_alpha(const Rec& r, double sx, double sy, double& dx,
                                           double& dy, float& oG, float& a) {
  dx = r.mx - sx;
  dy = r.my - sy;
  oG = __builtin_amdgcn_exp2f(rec_exponent(r, (float)dx, (float)dy));
  a = fminf(kAlphaMax, oG);
  return a >= kAlphaMin;
}

// DPP move with zero fill where the lane has no source or its row is masked.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, true));
}

// Sum over the wavefront, result in lane 63: xor 1 and xor 2 within quads,
// half-row and row mirrors (sums of 8 and 16), then row broadcasts of lanes
// 15 and 31 into the upper rows.  Every lane must be active.
__device__ __forceinline__ float wave_sum_to_last(float x) {
  x += dpp<0xB1>(x);        // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);        // quad_perm [2,3,0,1]
  x += dpp<0x141>(x);       // row_half_mirror
  x += dpp<0x140>(x);       // row_mirror
  x += dpp<0x142, 0xA>(x);  // row_bcast:15 -> rows 1 and 3
  x += dpp<0x143, 0xC>(x);  // row_bcast:31 -> rows 2 and 3
  return x;
}

// Sums of ten values over the wavefront, scattered: afterwards lane l of
// the first row holds the total of value rs_index(l) (lanes whose index is
// -1 hold nothing).  Four in-row halving steps -- each lane keeps half of
// its values and adds the partner's copy of that half: row mirror (partner
// differs in bit 3), half-row mirror (bit 2), quad reversal (bit 1), quad
// swap (bit 0) -- then the row pairs (bit 4) and half-waves (bit 5) are
// added with the gfx950 lane swaps.  37 VALU operations instead of the 60
// of ten separate reductions.  Every lane must be active.
__device__ __forceinline__ float sel(bool c, float a, float b) { return c ? a : b; }

__device__ __forceinline__ float reduce_scatter10(const float* g) {
  const int l = threadIdx.x & 15;
  const bool b3 = l & 8, b2 = l & 4, b1 = l & 2, b0 = l & 1;
  float h[6], u[4], w[2];
#pragma unroll
  for (int k = 0; k < 5; ++k)
    h[k] = sel(b3, g[k + 5], g[k]) + dpp<0x140>(sel(b3, g[k], g[k + 5]));  // row_mirror
  h[5] = 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    u[k] = sel(b2, h[k + 3], h[k]) + dpp<0x141>(sel(b2, h[k], h[k + 3]));  // row_half_mirror
  u[3] = 0.0f;
#pragma unroll
  for (int k = 0; k < 2; ++k)
    w[k] = sel(b1, u[k + 2], u[k]) + dpp<0x1B>(sel(b1, u[k], u[k + 2]));  // quad [3,2,1,0]
  float z = sel(b0, w[1], w[0]) + dpp<0xB1>(sel(b0, w[0], w[1]));         // quad [1,0,3,2]
  const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(z), __float_as_uint(z),
                                                    false, false);
  z = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(z), __float_as_uint(z),
                                                    false, false);
  return __uint_as_float(r32[0]) + __uint_as_float(r32[1]);
}

// Which of the ten values reduce_scatter10 leaves in lane l (first 16 lanes
// meaningful), -1 for none.
__device__ __forceinline__ int rs_index(int lane) {
  const int l = lane & 15;
  const int j = ((l & 2) ? 2 : 0) + (l & 1);       // index among u
  if (j >= 3) return -1;
  const int hidx = ((l & 4) ? 3 : 0) + j;          // index among h
  if (hidx >= 5) return -1;
  return ((l & 8) ? 5 : 0) + hidx;
}

template <int TW, int TH>
struct Tile {
  static constexpr int NPX = TW * TH;
  static constexpr int PPL = NPX / kWave;  // pixels per lane: 1, 2 or 4
  static __device__ __forceinline__ int x(int l, int k) {
    return PPL == 1 ? (l & 7) : 2 * (l & 7) + (k & 1);
  }
  static __device__ __forceinline__ int y(int l, int k) {
    return PPL == 4 ? 2 * (l >> 3) + (k >> 1) : (l >> 3);
  }
};

__device__ __forceinline__ int find_view(const ViewTable& vt, int gtile) {
  int v = 0;
  while (v + 1 < vt.n_views && gtile >= vt.v[v + 1].tile_off) ++v;
  return v;
}

// Records of a tile list: a copy in list order written by the per-tile
// binning, so that a batch is one contiguous, coalesced read, or (radix
// binning) gathered from the record array by record id.  fresh (a copy
// only): the records were written by this wavefront in this kernel, so they
// are read at device scope, past the vector L1 (which may hold an older copy
// of the line, loaded for a neighbouring tile).
__device__ __forceinline__ void stage(Rec* srec, uint32_t* sval, RecSrc lrec,
                                      const uint32_t* __restrict__ sorted_vals, uint32_t first,
                                      int count, int lane, bool fresh = false) {
  for (int k = lane; k < count; k += kWave) {
    uint64_t* dst = reinterpret_cast<uint64_t*>(srec + k);
    if (fresh) {
      const uint64_t* src = reinterpret_cast<const uint64_t*>(lrec.base + first + k);
      uint64_t w[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        w[q] = __hip_atomic_load(src + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int q = 0; q < 8; ++q) dst[q] = w[q];
    } else {
      const float4* src = reinterpret_cast<const float4*>(lrec.at(first + k));
      float4* d4 = reinterpret_cast<float4*>(dst);
      const float4 a0 = src[0], a1 = src[1], a2 = src[2], a3 = src[3];
      d4[0] = a0; d4[1] = a1; d4[2] = a2; d4[3] = a3;
    }
    if (sval) sval[k] = sorted_vals[first + k];
  }
}

// ------------------------------------------------------------------ forward
// Splats per step of the forward's compositing loop.
constexpr int kFwdSplats = 4;
template <int TW, int TH, bool CKPT>
__device__ __forceinline__ void fwd_tile(int gtile, RecSrc lrec,
                                         const uint32_t* __restrict__ ranges,
                                         const float* __restrict__ cams, const ViewTable& vt,
                                         int B, float* __restrict__ color,
                                         float* __restrict__ depth, float* __restrict__ T_final,
                                         uint32_t* __restrict__ last,
                                         uint32_t* __restrict__ tile_last,
                                         const float* __restrict__ target_rgb,
                                         const float* __restrict__ target_depth,
                                         float* __restrict__ tile_loss,
                                         const uint32_t* __restrict__ boff,
                                         float* __restrict__ ckpt, Rec* srec,
                                         const TileList* known = nullptr) {
  using TG = Tile<TW, TH>;
  constexpr int PPL = TG::PPL;
  constexpr int NPX = TG::NPX;
  const int v = find_view(vt, gtile);
  const ViewInfo vi = vt.v[v];
  const int lt = gtile - vi.tile_off;
  const int tx0 = (lt % vi.tiles_x) * TW, ty0 = (lt / vi.tiles_x) * TH;
  const int lane = threadIdx.x;
  // the list: from the binning's ranges, or from this wavefront's own sort
  // (range in registers, records possibly staged already)
  const uint32_t s = known ? known->start : ranges[2 * (int64_t)gtile];
  const uint32_t e = known ? known->end : ranges[2 * (int64_t)gtile + 1];
  const bool fresh = known && known->fresh, staged = known && known->staged;
  // the long lists start first (work order) and end last: their wavefronts
  // take precedence at instruction issue over the short tiles sharing a SIMD
  if (e - s >= (uint32_t)kWave) __builtin_amdgcn_s_setprio(2);

  double sx[PPL], sy[PPL];
  float T[PPL], c0[PPL], c1[PPL], c2[PPL], D[PPL];
  uint32_t lastpos[PPL];
  bool done[PPL], inside[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int px = tx0 + TG::x(lane, k), py = ty0 + TG::y(lane, k);
    inside[k] = (px < vi.W) && (py < vi.H);
    sx[k] = px + 0.5;
    sy[k] = py + 0.5;

    T[k] = 1.0f; c0[k] = c1[k] = c2[k] = D[k] = 0.0f;
    lastpos[k] = 0;
    done[k] = !inside[k];
  }
  auto active = [&]() {
    bool a = false;
#pragma unroll
    for (int k = 0; k < PPL; ++k) a = a || !done[k];
    return a;
  };
  bool more = true;
  for (uint32_t b = s; more && b < e; b += (uint32_t)B) {
    if (ballot64(active()) == 0) break;
    const int nb = (int)min((uint32_t)B, e - b);
    if (!(staged && b == s)) {  // the sort staged the first batch
      __syncthreads();
      stage(srec, nullptr, lrec, nullptr, b, nb, lane, fresh);
      __syncthreads();
    }
    // segments between the 64-position bucket boundaries of the list, so
    // that the pixel states are stored outside the per-splat loop
    for (int j = 0; more && j < nb;) {
      const uint32_t q0 = b - s + (uint32_t)j;
      if constexpr (CKPT) {
        // state of every pixel before each 64th splat of the tile list (the
        // state before the first splat is the empty one and is not stored)
        if (q0 != 0 && (q0 & (kBucket - 1)) == 0) {
          float* cp = ckpt + (int64_t)(boff[gtile] + q0 / kBucket) * (kStateFloats * NPX);
#pragma unroll
          for (int k = 0; k < PPL; ++k) {
            const int jj = TG::y(lane, k) * TW + TG::x(lane, k);
            cp[jj] = T[k];
            cp[NPX + jj] = c0[k];
            cp[2 * NPX + jj] = c1[k];
            cp[3 * NPX + jj] = c2[k];
            cp[4 * NPX + jj] = D[k];
          }
        }
      }
      const int jend = min(nb, j + (int)(kBucket - (q0 & (kBucket - 1))));
      for (; j < jend; j += kFwdSplats) {
        // kFwdSplats records at once (whole records, broadcast LDS reads):
        // their alphas are independent, only the blends are ordered.  Every
        // decision of eval_alpha is a select: no divergent branches.
        constexpr int NS = kFwdSplats;
        Rec rr[NS];
        bool hasu[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
          hasu[u] = j + u < jend;
          rr[u] = srec[hasu[u] ? j + u : j];
        }
        const uint32_t pos0 = b - s + (uint32_t)j + 1u;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
          float au[NS];
#pragma unroll
          for (int u = 0; u < NS; ++u) {
            const double dx = rr[u].mx - sx[k], dy = rr[u].my - sy[k];
            au[u] = fminf(kAlphaMax,
                          __builtin_amdgcn_exp2f(rec_exponent(rr[u], (float)dx, (float)dy)));
          }
          // a splat that is not blended gets weight 0: colour, depth are
          // non-negative and finite, so fma(x, 0, acc) leaves acc as it is
          // and one select replaces four
#pragma unroll
          for (int u = 0; u < NS; ++u) {
            const bool hit = hasu[u] && !done[k] && au[u] >= kAlphaMin;
            const float w0 = au[u] * T[k];
            const float Tn = T[k] - w0;  // T (1 - alpha)
            const bool stop = Tn < kTMin;
            const bool blend = hit && !stop;
            const float w = blend ? w0 : 0.0f;
            c0[k] = fmaf(rr[u].r, w, c0[k]);
            c1[k] = fmaf(rr[u].g, w, c1[k]);
            c2[k] = fmaf(rr[u].b, w, c2[k]);
            D[k] = fmaf(rr[u].z, w, D[k]);
            T[k] -= w;
            lastpos[k] = blend ? pos0 + (uint32_t)u : lastpos[k];
            done[k] = done[k] || (hit && stop);
          }
        }
        if (ballot64(active()) == 0) {
          more = false;
          break;
        }
      }
      // the next segment starts at jend, whatever the step: a step of
      // kFwdSplats may pass it (its splats past jend are masked off)
      if (more) j = jend;
    }
  }
  const float* cam = cams + (int64_t)v * GS_CAMERA_FLOATS;
  const float bg0 = cam[17], bg1 = cam[18], bg2 = cam[19];
  const int64_t npx = (int64_t)vi.W * vi.H;
  float lrgb = 0.0f, ld = 0.0f;
  uint32_t lmax = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    lmax = max(lmax, lastpos[k]);
    if (!inside[k]) continue;
    const int px = tx0 + TG::x(lane, k), py = ty0 + TG::y(lane, k);
    const int64_t pl = (int64_t)py * vi.W + px;
    const int64_t pix = (int64_t)vi.pix_off + pl;
    const int64_t cbase = 3 * (int64_t)vi.pix_off + pl;
    const float o0 = fmaf(T[k], bg0, c0[k]), o1 = fmaf(T[k], bg1, c1[k]), o2 = fmaf(T[k], bg2, c2[k]);
    color[cbase] = o0;
    color[cbase + npx] = o1;
    color[cbase + 2 * npx] = o2;
    depth[pix] = D[k];
    T_final[pix] = T[k];
    last[pix] = lastpos[k];
    if (target_rgb) {
      lrgb += fabsf(o0 - target_rgb[cbase]) + fabsf(o1 - target_rgb[cbase + npx]) +
              fabsf(o2 - target_rgb[cbase + 2 * npx]);
      if (target_depth) ld += fabsf(D[k] - target_depth[pix]);
    }
  }
  const uint32_t m = wave_max(lmax);
  if (target_rgb) {
    lrgb = wave_sum_to_last(lrgb);
    ld = wave_sum_to_last(ld);
  }
  if (lane == kWave - 1) {
    tile_last[gtile] = m;
    if (target_rgb) {
      tile_loss[2 * (int64_t)gtile] = lrgb;
      tile_loss[2 * (int64_t)gtile + 1] = ld;
    }
  }
}

template <int TW, int TH, bool CKPT>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(TW * TH == 64 ? 7 : 1))) k_render_fwd(
    RecSrc lrec,
    const uint32_t* __restrict__ ranges, const float* __restrict__ cams, ViewTable vt, int B,
    float* __restrict__ color, float* __restrict__ depth, float* __restrict__ T_final,
    uint32_t* __restrict__ last, uint32_t* __restrict__ tile_last,
    const float* __restrict__ target_rgb, const float* __restrict__ target_depth,
    float* __restrict__ tile_loss, const uint32_t* __restrict__ order,
    int32_t* __restrict__ queue, int chunk, const uint32_t* __restrict__ boff,
    float* __restrict__ ckpt, TileSortArgs sort) {
  extern __shared__ __align__(16) unsigned char smem[];
  Rec* srec = reinterpret_cast<Rec*>(smem);
  // With sort.cnt set (a whole iteration), the wavefront first sorts its
  // tile's list (lists of at most kTileSortSmall pairs; longer ones are
  // sorted already), in the same LDS; the barrier makes the sorted records
  // and the range visible to every lane before the compositing reads them.
  auto tile = [&](int g) {
    if (sort.cnt) {
      // the list's first B records are staged by the sort itself
      const TileList L = sort_tile_wave(sort, g, (int)threadIdx.x,
                                        reinterpret_cast<uint64_t*>(smem), srec, B);
      __syncthreads();
      fwd_tile<TW, TH, CKPT>(g, lrec, ranges, cams, vt, B, color, depth, T_final, last,
                             tile_last, target_rgb, target_depth, tile_loss, boff, ckpt, srec,
                             &L);
      return;
    }
    fwd_tile<TW, TH, CKPT>(g, lrec, ranges, cams, vt, B, color, depth, T_final, last,
                           tile_last, target_rgb, target_depth, tile_loss, boff, ckpt, srec);
  };
  if (queue == nullptr) {
    tile(order ? (int)order[blockIdx.x] : (int)blockIdx.x);
    return;
  }
  // persistent: chunks of `chunk` tiles of the work order, taken with a
  // static stride (the order is longest first, so the first round takes the
  // longest tiles; no shared counter)
  const int n_items = (vt.total_tiles + chunk - 1) / chunk;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int first = item * chunk;
    const int lastt = min(vt.total_tiles, first + chunk);
    for (int k = first; k < lastt; ++k) {
      __syncthreads();  // the LDS of the previous tile is reused
      tile(order ? (int)order[k] : k);
    }
  }
}

// Per-view L1 loss from the per-tile sums, in a fixed order.
constexpr int kLossThreads = kLossVirtual;
__global__ void __launch_bounds__(kLossThreads) k_loss_reduce(const float* __restrict__ tile_loss,
                                                              ViewTable vt, float lambda_depth,
                                                              int has_depth, float* __restrict__ loss) {
  const int v = blockIdx.x;
  const ViewInfo vi = vt.v[v];
  loss_reduce_view<kLossThreads>(reinterpret_cast<const float2*>(tile_loss) + vi.tile_off,
                                 vi.tiles_x * vi.tiles_y, (double)vi.W * vi.H, lambda_depth,
                                 has_depth, loss + v);
}

// ------------------------------------------------------------------ backward
template <int TW, int TH>
__device__ __forceinline__ void bwd_tile(
    int gtile, RecSrc lrec,
    const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ tile_last, const float* __restrict__ cams, const ViewTable& vt,
    int B, const float* __restrict__ color, const float* __restrict__ depth,
    const float* __restrict__ T_final, const uint32_t* __restrict__ last,
    const float* __restrict__ dL_dcolor, const float* __restrict__ dL_ddepth,
    const float* __restrict__ target_rgb, const float* __restrict__ target_depth, int fused,
    float lambda_depth, float* __restrict__ grad_pair, Rec* srec, uint32_t* sval) {
  using TG = Tile<TW, TH>;
  constexpr int PPL = TG::PPL;
  const int v = find_view(vt, gtile);
  const ViewInfo vi = vt.v[v];
  const int lt = gtile - vi.tile_off;
  const int tx0 = (lt % vi.tiles_x) * TW, ty0 = (lt / vi.tiles_x) * TH;
  const int lane = threadIdx.x;
  const uint32_t s = ranges[2 * (int64_t)gtile], e = ranges[2 * (int64_t)gtile + 1];
  const uint32_t tl = tile_last[gtile];
  const float* cam = cams + (int64_t)v * GS_CAMERA_FLOATS;
  const float bg0 = cam[17], bg1 = cam[18], bg2 = cam[19];

  // pairs beyond the last used position get zero gradients
  for (uint32_t k = tl + (uint32_t)lane; k < e - s; k += kWave) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    store_pair(grad_pair, sorted_vals[s + k], z, z, make_float2(0.f, 0.f));
  }

  // lanes of the first row write the scattered sums of the ten partials;
  // the conic and mean entries carry their sign and halves here
  const int my_idx = lane < 16 ? rs_index(lane) : -1;
  const float my_scale = (my_idx == 5 || my_idx == 7) ? -0.5f : (my_idx >= 6 ? -1.0f : 1.0f);
  double sx[PPL], sy[PPL];
  float T[PPL], gC0[PPL], gC1[PPL], gC2[PPL], gD[PPL], Sc0[PPL], Sc1[PPL], Sc2[PPL], Sd[PPL];
  uint32_t L[PPL];
  const int64_t npx = (int64_t)vi.W * vi.H;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int px = tx0 + TG::x(lane, k), py = ty0 + TG::y(lane, k);
    sx[k] = px + 0.5;
    sy[k] = py + 0.5;
    T[k] = 1.0f; gC0[k] = gC1[k] = gC2[k] = gD[k] = 0.0f;
    L[k] = 0;
    if (px < vi.W && py < vi.H) {
      const int64_t pl = (int64_t)py * vi.W + px;
      const int64_t pix = (int64_t)vi.pix_off + pl;
      const int64_t cbase = 3 * (int64_t)vi.pix_off + pl;
      T[k] = T_final[pix];
      L[k] = last[pix];
      if (fused) {
        const float inv3 = 1.0f / (3.0f * (float)npx);
        const float d0 = color[cbase] - target_rgb[cbase];
        const float d1 = color[cbase + npx] - target_rgb[cbase + npx];
        const float d2 = color[cbase + 2 * npx] - target_rgb[cbase + 2 * npx];
        gC0[k] = d0 > 0.0f ? inv3 : (d0 < 0.0f ? -inv3 : 0.0f);
        gC1[k] = d1 > 0.0f ? inv3 : (d1 < 0.0f ? -inv3 : 0.0f);
        gC2[k] = d2 > 0.0f ? inv3 : (d2 < 0.0f ? -inv3 : 0.0f);
        if (target_depth) {
          const float dd = depth[pix] - target_depth[pix];
          const float sc = lambda_depth / (float)npx;
          gD[k] = dd > 0.0f ? sc : (dd < 0.0f ? -sc : 0.0f);
        }
      } else {
        gC0[k] = dL_dcolor[cbase];
        gC1[k] = dL_dcolor[cbase + npx];
        gC2[k] = dL_dcolor[cbase + 2 * npx];
        gD[k] = dL_ddepth ? dL_ddepth[pix] : 0.0f;
      }
    }
    // behind-sums: background seen through T_final, nothing behind in depth
    Sc0[k] = T[k] * bg0;
    Sc1[k] = T[k] * bg1;
    Sc2[k] = T[k] * bg2;
    Sd[k] = 0.0f;
  }

  for (int bend = (int)tl; bend > 0; bend -= B) {
    const int bstart = max(0, bend - B);
    const int nb = bend - bstart;
    __syncthreads();
    stage(srec, sval, lrec, sorted_vals, s + (uint32_t)bstart, nb, lane);
    __syncthreads();
#pragma unroll 2
    for (int j = nb - 1; j >= 0; --j) {
      const uint32_t pos = (uint32_t)(bstart + j);
      const Rec& r = srec[j];
      float ca, cb, cc;
      rec_conic(r, ca, cb, cc);
      float g[10];
#pragma unroll
      for (int f = 0; f < 10; ++f) g[f] = 0.0f;
      bool contrib = false;
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        if (pos < L[k]) {
          double dx, dy;
          float oG, a;
          if (eval_alpha(r, sx[k], sy[k], dx, dy, oG, a)) {
            contrib = true;
            const float inv_om = __builtin_amdgcn_rcpf(1.0f - a);
            const float Tk = T[k] * inv_om;
            const float wgt = a * Tk;
            g[0] = fmaf(wgt, gC0[k], g[0]);
            g[1] = fmaf(wgt, gC1[k], g[1]);
            g[2] = fmaf(wgt, gC2[k], g[2]);
            g[3] = fmaf(wgt, gD[k], g[3]);
            const float front = gC0[k] * r.r + gC1[k] * r.g + gC2[k] * r.b + gD[k] * r.z;
            const float behind = gC0[k] * Sc0[k] + gC1[k] * Sc1[k] + gC2[k] * Sc2[k] + gD[k] * Sd[k];
            const float g_alpha = Tk * front - behind * inv_om;
            Sc0[k] = fmaf(r.r, wgt, Sc0[k]);
            Sc1[k] = fmaf(r.g, wgt, Sc1[k]);
            Sc2[k] = fmaf(r.b, wgt, Sc2[k]);
            Sd[k] = fmaf(r.z, wgt, Sd[k]);
            T[k] = Tk;
            // unclamped alpha only (no gradient through the 0.99 clamp);
            // the conic and mean partials are formed from t = gpow dx,
            // u = gpow dy, their signs and halves applied after the sum
            const bool open = oG <= kAlphaMax;
            const float gpow = open ? a * g_alpha : 0.0f;
            const float fx = (float)dx, fy = (float)dy;
            const float t = gpow * fx, u = gpow * fy;
            g[4] += gpow;  // (divided by the opacity at the store)
            g[5] = fmaf(t, fx, g[5]);
            g[6] = fmaf(t, fy, g[6]);
            g[7] = fmaf(u, fy, g[7]);
            g[8] = fmaf(ca, t, fmaf(cb, u, g[8]));
            g[9] = fmaf(cb, t, fmaf(cc, u, g[9]));
          }
        }
      }
      float* gpf = grad_pair + (int64_t)sval[j] * kPairGrad;
      if (ballot64(contrib) != 0) {
        const float z = reduce_scatter10(g);
        const float sc = my_idx == 4 ? (r.o > 0.0f ? 1.0f / r.o : 0.0f) : my_scale;
        if (my_idx >= 0) gpf[my_idx] = z * sc;
      } else if (lane == 0) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        store_pair(gpf, 0, z, z, make_float2(0.f, 0.f));
      }
    }
  }
}

template <int TW, int TH>
__global__ void __launch_bounds__(kWave) k_render_bwd(
    RecSrc lrec,
    const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ tile_last, const float* __restrict__ cams, ViewTable vt, int B,
    const float* __restrict__ color, const float* __restrict__ depth,
    const float* __restrict__ T_final, const uint32_t* __restrict__ last,
    const float* __restrict__ dL_dcolor, const float* __restrict__ dL_ddepth,
    const float* __restrict__ target_rgb, const float* __restrict__ target_depth, int fused,
    float lambda_depth, float* __restrict__ grad_pair, const uint32_t* __restrict__ order,
    int32_t* __restrict__ queue, int chunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  Rec* srec = reinterpret_cast<Rec*>(smem);
  uint32_t* sval = reinterpret_cast<uint32_t*>(smem + (size_t)B * sizeof(Rec));
  if (queue == nullptr) {
    const int g = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    bwd_tile<TW, TH>(g, lrec, sorted_vals, ranges, tile_last, cams, vt, B, color, depth,
                     T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused,
                     lambda_depth, grad_pair, srec, sval);
    return;
  }
  const int n_items = (vt.total_tiles + chunk - 1) / chunk;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int first = item * chunk;
    const int lastt = min(vt.total_tiles, first + chunk);
    for (int k = first; k < lastt; ++k) {
      const int g = order ? (int)order[k] : k;
      bwd_tile<TW, TH>(g, lrec, sorted_vals, ranges, tile_last, cams, vt, B, color,
                       depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth,
                       fused, lambda_depth, grad_pair, srec, sval);
    }
  }
}

// ----------------------------------------------------- splat-wise backward
// Sec. III-C-1 / Fig. 4a mapped to wave64.  The tile list is cut into
// buckets of 64 consecutive splats; one wavefront takes a bucket and lane l
// owns its l-th splat.  The forward stored each pixel's state X = (T, RGB,
// D) before every 64th splat, so a bucket starts from stored states and
// needs nothing from the other buckets of its tile: buckets are the unit of
// parallelism, which also splits long tile lists over many wavefronts.
//
// All lanes of a segment take the same pixel at each step.  Lane l
// evaluates its splat's alpha with the forward's code (the same bits, so
// the same skip decisions; the forward's stop rule is its stored last
// position).  What lies in front of lane l's splat at the pixel is the
// segment's stored state advanced over the blended splats of lanes < l: the
// transmittance is T_in times the product of (1 - alpha) over those lanes
// (the inclusive prefix product divided by the lane's own factor), and the
// front part of the loss-weighted output Q = gC . C + gD . D an inclusive
// prefix sum of alpha T gC . c, both taken across the lanes with DPP.  What lies behind the splat is the final pixel minus the front part,
// P - Q with P = gC . (colour output) + gD . (depth output).  A bucket thus
// costs one step per pixel, with no pipeline to fill or drain.  Each lane
// accumulates its own splat's ten partial gradients over the tile's pixels
// and writes them once: no reduction over lanes and no atomics.
//
// Buckets with at most 32 pairs share a wavefront: each 32-lane half runs
// its own bucket (the scans stop at the half), two buckets per NPX steps.
// The binning queues buckets by size (more than 32 pairs / at most 32).

// Inclusive product / sum over segments of SEG (64 or 32) lanes, in place,
// of two independent values at once (two pixels): steps in rows of 16
// (row_shr 1, 2, 4, 8), then the ends of rows 0 and 2 into rows 1 and 3
// (row_bcast:15), and for 64 lanes the end of row 1 into rows 2 and 3
// (row_bcast:31).  Each step is one DPP multiply or add whose lanes
// without a source (or outside the row mask) are not written, i.e. keep
// their value.  A DPP read of a VGPR written by the previous VALU
// instruction needs two wait states: the two scans' steps alternate, so
// one wait state plus the other scan's step covers it (two before the
// first step, whose inputs the compiler's code has just written).
#define GS_DPP2(OP, CTRL) OP " %0, %0, %0 " CTRL " bank_mask:0xf\n\t" OP " %1, %1, %1 " CTRL " bank_mask:0xf\n\t"
#define GS_SEG_SCAN32_2(OP)                                          \
  "s_nop 1\n\t" GS_DPP2(OP, "row_shr:1 row_mask:0xf")              \
  "s_nop 0\n\t" GS_DPP2(OP, "row_shr:2 row_mask:0xf")              \
  "s_nop 0\n\t" GS_DPP2(OP, "row_shr:4 row_mask:0xf")              \
  "s_nop 0\n\t" GS_DPP2(OP, "row_shr:8 row_mask:0xf")              \
  "s_nop 0\n\t" GS_DPP2(OP, "row_bcast:15 row_mask:0xa")
template <int SEG>
__device__ __forceinline__ void seg_scan_mul2(float& x, float& y) {
  if (SEG == 64)
    asm volatile(GS_SEG_SCAN32_2("v_mul_f32_dpp") "s_nop 0\n\t"
                 GS_DPP2("v_mul_f32_dpp", "row_bcast:31 row_mask:0xc") : "+v"(x), "+v"(y));
  else
    asm volatile(GS_SEG_SCAN32_2("v_mul_f32_dpp") : "+v"(x), "+v"(y));
}
template <int SEG>
__device__ __forceinline__ void seg_scan_add2(float& x, float& y) {
  if (SEG == 64)
    asm volatile(GS_SEG_SCAN32_2("v_add_f32_dpp") "s_nop 0\n\t"
                 GS_DPP2("v_add_f32_dpp", "row_bcast:31 row_mask:0xc") : "+v"(x), "+v"(y));
  else
    asm volatile(GS_SEG_SCAN32_2("v_add_f32_dpp") : "+v"(x), "+v"(y));
}
#undef GS_SEG_SCAN32_2
#undef GS_DPP2

template <int TW, int TH, int SEG>
__device__ __forceinline__ void splat_wave(
    const uint2* __restrict__ queue, uint32_t q_first, uint32_t q_count,
    RecSrc lrec,
    const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ tile_last, const uint32_t* __restrict__ boff,
    const float* __restrict__ ckpt, const ViewTable& vt, const float* __restrict__ color,
    const float* __restrict__ depth, const uint32_t* __restrict__ last,
    const float* __restrict__ dL_dcolor, const float* __restrict__ dL_ddepth,
    const float* __restrict__ target_rgb, const float* __restrict__ target_depth, int fused,
    float lambda_depth, float* __restrict__ grad_pair, float4* pxa, float4* pxb, double2* pxc) {
  static_assert(SEG == 64 || SEG == 32, "segment of 64 or 32 lanes");
  constexpr int NPX = TW * TH;
  constexpr int LOG_TW = TW == 16 ? 4 : 3;
  const int lane = threadIdx.x;
  const int seg = SEG == 64 ? 0 : lane >> 5, ls = lane & (SEG - 1);
  const uint32_t qi = q_first + (uint32_t)seg;
  const bool has = qi < q_count;
  const uint2 ent = has ? queue[qi] : make_uint2(0u, 0u);
  const int gtile = (int)ent.x;
  const uint32_t k = ent.y;
  uint32_t s = 0, npairs = 0, tl = 0;
  if (has) {
    s = ranges[2 * (int64_t)gtile];
    npairs = ranges[2 * (int64_t)gtile + 1] - s;
    tl = tile_last[gtile];
  }
  const uint32_t q0 = k * kBucket;
  const uint32_t pos = q0 + (uint32_t)ls;
  const bool live = has && pos < tl;
  if (has && pos < npairs && !live) {  // pairs behind the last used position: zero gradient
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    store_pair(grad_pair, sorted_vals[s + pos], z, z, make_float2(0.f, 0.f));
  }
  const bool active = has && q0 < tl;  // uniform over the segment
  if (ballot64(active) == 0) return;   // uniform

  const int v = active ? find_view(vt, gtile) : 0;
  const ViewInfo vi = vt.v[v];
  const int lt = gtile - vi.tile_off;
  const int tx0 = (lt % vi.tiles_x) * TW, ty0 = (lt / vi.tiles_x) * TH;
  const int64_t npx = (int64_t)vi.W * vi.H;
  float4* sa = pxa + seg * NPX;
  float4* sb = pxb + seg * NPX;
  double2* sc = pxc + seg * NPX;  // sample point of each pixel

  // pixel table of the segment's tile: loss gradients, P, last position,
  // stored state (T, Q), kept only for the pixels whose last position lies
  // past the bucket's first splat.  At any other pixel no lane of the bucket
  // is blended, so every term it adds is zero: the table holds the others
  // in pixel order, and the loop below runs over them alone.
  const uint64_t segmask = SEG == 64 ? ~0ull : (0xFFFFFFFFull << (32 * seg));
  const uint64_t below = lanemask_lt() & segmask;
  uint32_t kept = 0;
  for (int j = ls; j < NPX; j += SEG) {  // (NPX is a multiple of SEG: uniform)
    const int px = tx0 + (j & (TW - 1)), py = ty0 + (j >> LOG_TW);
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = make_float4(0.f, 0.f, 1.f, 0.f);
    bool keep = false;
    if (active && px < vi.W && py < vi.H) {
      const float* cp = ckpt + (int64_t)(boff[gtile] + k) * (kStateFloats * NPX);
      const int64_t pl = (int64_t)py * vi.W + px;
      const int64_t pix = (int64_t)vi.pix_off + pl;
      const int64_t cbase = 3 * (int64_t)vi.pix_off + pl;
      const float o0 = color[cbase], o1 = color[cbase + npx], o2 = color[cbase + 2 * npx];
      const float od = depth[pix];
      if (fused) {
        const float inv3 = 1.0f / (3.0f * (float)npx);
        const float d0 = o0 - target_rgb[cbase];
        const float d1 = o1 - target_rgb[cbase + npx];
        const float d2 = o2 - target_rgb[cbase + 2 * npx];
        a.x = d0 > 0.0f ? inv3 : (d0 < 0.0f ? -inv3 : 0.0f);
        a.y = d1 > 0.0f ? inv3 : (d1 < 0.0f ? -inv3 : 0.0f);
        a.z = d2 > 0.0f ? inv3 : (d2 < 0.0f ? -inv3 : 0.0f);
        if (target_depth) {
          const float dd = od - target_depth[pix];
          const float sc = lambda_depth / (float)npx;
          a.w = dd > 0.0f ? sc : (dd < 0.0f ? -sc : 0.0f);
        }
      } else {
        a.x = dL_dcolor[cbase];
        a.y = dL_dcolor[cbase + npx];
        a.z = dL_dcolor[cbase + 2 * npx];
        a.w = dL_ddepth ? dL_ddepth[pix] : 0.0f;
      }
      b.x = a.x * o0 + a.y * o1 + a.z * o2 + a.w * od;
      const uint32_t lp = last[pix];
      b.y = __uint_as_float(lp);
      keep = lp > q0;
      if (keep && k > 0) {  // the first bucket starts from T = 1 and nothing accumulated
        b.z = cp[j];
        b.w = a.x * cp[NPX + j] + a.y * cp[2 * NPX + j] + a.z * cp[3 * NPX + j] + a.w * cp[4 * NPX + j];
      }
    }
    const uint64_t m = ballot64(keep) & segmask;
    if (keep) {
      const uint32_t e = kept + (uint32_t)__popcll(m & below);
      sa[e] = a;
      sb[e] = make_float4(b.x - b.w, b.y, b.z, 0.0f);  // (P - Q_in, last, T_in)
      sc[e] = make_double2((double)px + 0.5, (double)py + 0.5);
    }
    kept += (uint32_t)__popcll(m);
  }
  // two half-wave segments step together, two pixels a step: a table with
  // fewer entries is padded with pixels at which nothing is blended (last = 0)
  const uint32_t most = SEG == 64 ? kept : max(kept, (uint32_t)__shfl_xor((int)kept, 32));
  const uint32_t steps = (most + 1u) & ~1u;
  for (uint32_t e = kept + (uint32_t)ls; e < steps; e += SEG) {
    sa[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    sb[e] = make_float4(0.f, 0.f, 1.f, 0.f);
    sc[e] = make_double2(0.5, 0.5);
  }
  const int nsteps = __builtin_amdgcn_readfirstlane((int)steps);
  __builtin_assume((nsteps & 1) == 0);
  __syncthreads();

  Rec r;
  if (live) {
    const float4* src = reinterpret_cast<const float4*>(lrec.at(s + pos));
    float4* dst = reinterpret_cast<float4*>(&r);
    dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3];
  } else {
    r.mx = r.my = 0.0;
    r.t = r.s1 = r.s2 = r.lo = 0.0f;
    r.o = r.z = r.r = r.g = r.b = 0.0f;
    r.clamp = r.pad[0] = r.pad[1] = 0u;
  }
  float ca, cb, cc;
  rec_conic(r, ca, cb, cc);
  float g[10];
#pragma unroll
  for (int f = 0; f < 10; ++f) g[f] = 0.0f;
  // two pixels per iteration (the step count is even), their scans
  // interleaved; each lane accumulates pixel j before pixel j + 1
  for (int j = 0; j < nsteps; j += 2) {
    float4 b[2], gc[2];
    float dxf[2], dyf[2], oG[2], a[2], inv_om[2], f[2];
    bool hit[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      b[u] = sb[j + u];  // P - Q_in, last, T_in of the segment's kept pixel
      const double2 sxy = sc[j + u];
      // alpha as in the forward (same bits)
      dxf[u] = (float)(r.mx - sxy.x);
      dyf[u] = (float)(r.my - sxy.y);
      oG[u] = __builtin_amdgcn_exp2f(rec_exponent(r, dxf[u], dyf[u]));
      a[u] = fminf(kAlphaMax, oG[u]);
      // (no short-circuit: every term is evaluated, so nothing branches; no
      // early exit when no lane is blended at a pixel: rare, and its test
      // costs two VALU per step)
      hit[u] = live & (pos < __float_as_uint(b[u].y)) & (a[u] >= kAlphaMin);
      gc[u] = sa[j + u];
      // alpha of a blended splat, 0 otherwise: its 1 - alpha is the scan's
      // factor and alpha T the blend weight, with no further selects
      a[u] = hit[u] ? a[u] : 0.0f;
      f[u] = 1.0f - a[u];
      inv_om[u] = __builtin_amdgcn_rcpf(f[u]);
    }
    // transmittance in front of the splat: the segment's inclusive product
    // over its blended splats with the lane's own factor taken out again
    // (read by blended lanes only, whose factor 1 - alpha >= 0.01)
    seg_scan_mul2<SEG>(f[0], f[1]);
    float Tl[2], wgt[2], front[2], q[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      Tl[u] = (b[u].z * f[u]) * inv_om[u];
      wgt[u] = a[u] * Tl[u];
      front[u] = fmaf(gc[u].w, r.z, fmaf(gc[u].z, r.b, fmaf(gc[u].y, r.g, gc[u].x * r.r)));
      q[u] = wgt[u] * front[u];
    }
    seg_scan_add2<SEG>(q[0], q[1]);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      // behind the splat: P - (Q_in + the front part after the splat)
      const float g_alpha = fmaf(-(b[u].x - q[u]), inv_om[u], Tl[u] * front[u]);
      g[0] = fmaf(wgt[u], gc[u].x, g[0]);
      g[1] = fmaf(wgt[u], gc[u].y, g[1]);
      g[2] = fmaf(wgt[u], gc[u].z, g[2]);
      g[3] = fmaf(wgt[u], gc[u].w, g[3]);
      // moments of gpow = dL/dpower = alpha dL/dalpha (unclamped splats) and
      // of t = gpow dx, u = gpow dy; the opacity, conic and mean partials are
      // formed from them once, after the pixels (dL/do = sum gpow / o)
      const bool open = hit[u] & (oG[u] <= kAlphaMax);
      const float gpow = open ? a[u] * g_alpha : 0.0f;
      const float t = gpow * dxf[u], v = gpow * dyf[u];
      g[4] += gpow;
      g[5] = fmaf(t, dxf[u], g[5]);
      g[6] = fmaf(t, dyf[u], g[6]);
      g[7] = fmaf(v, dyf[u], g[7]);
      g[8] += t;
      g[9] += v;
    }
  }
  if (live) {
    store_pair(grad_pair, sorted_vals[s + pos], make_float4(g[0], g[1], g[2], g[3]),
               make_float4(r.o > 0.0f ? g[4] / r.o : 0.0f, -0.5f * g[5], -g[6], -0.5f * g[7]),
               make_float2(-(ca * g[8] + cb * g[9]), -(cb * g[8] + cc * g[9])));
  }
  __syncthreads();  // the pixel tables are rewritten by the next wave's work
}

// Grid-stride over the work of the two queues: one bucket per wave from
// the first, two per wave from the second.
template <int TW, int TH>
__global__ void __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(TW * TH == 64 ? 6 : 1))) k_render_bwd_splat(
    RecSrc lrec,
    const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ tile_last, const uint32_t* __restrict__ boff,
    const float* __restrict__ ckpt, const uint2* __restrict__ bq, int64_t bq_stride,
    const int32_t* __restrict__ fl, ViewTable vt, const float* __restrict__ color,
    const float* __restrict__ depth, const uint32_t* __restrict__ last,
    const float* __restrict__ dL_dcolor, const float* __restrict__ dL_ddepth,
    const float* __restrict__ target_rgb, const float* __restrict__ target_depth, int fused,
    float lambda_depth, float* __restrict__ grad_pair) {
  __shared__ float4 pxa[2 * TW * TH], pxb[2 * TW * TH];
  __shared__ double2 pxc[2 * TW * TH];
  const uint32_t q_full = (uint32_t)fl[F_BQ_FULL], q_half = (uint32_t)fl[F_BQ_HALF];
  const uint32_t w_full = q_full, w_half = (q_half + 1) / 2;
  for (uint32_t wv = blockIdx.x; wv < w_full + w_half; wv += gridDim.x) {
    if (wv < w_full)
      splat_wave<TW, TH, 64>(bq, wv, q_full, lrec, sorted_vals, ranges, tile_last,
                             boff, ckpt, vt, color, depth, last, dL_dcolor, dL_ddepth, target_rgb,
                             target_depth, fused, lambda_depth, grad_pair, pxa, pxb, pxc);
    else
      splat_wave<TW, TH, 32>(bq + bq_stride, 2 * (wv - w_full), q_half, lrec,
                         sorted_vals, ranges, tile_last, boff, ckpt, vt, color, depth, last,
                         dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, lambda_depth,
                         grad_pair, pxa, pxb, pxc);
  }
}

// The radix binning writes no record copy: its lists name their records.
RecSrc rec_src(const Plan& P, void* ws) {
  if (P.cfg.flags & GS_RADIX_BIN)
    return RecSrc{ws_at<Rec>(ws, P.off_rec), ws_at<uint32_t>(ws, P.off_sorted_rec)};
  return RecSrc{ws_at<Rec>(ws, P.off_srec), nullptr};
}

template <int TW, int TH>
hipError_t bwd_splat_launch(const Plan& P, void* ws, const float* cams, const float* color,
                            const float* depth, const uint32_t* last, const float* dL_dcolor,
                            const float* dL_ddepth, const float* target_rgb,
                            const float* target_depth, int fused, const uint32_t* sorted_vals,
                            int grid, hipStream_t s) {
  (void)cams;
  hipLaunchKernelGGL((k_render_bwd_splat<TW, TH>), dim3(grid), dim3(kWave), 0, s,
                     rec_src(P, ws), sorted_vals,
                     ws_at<uint32_t>(ws, P.off_ranges), ws_at<uint32_t>(ws, P.off_tile_last),
                     ws_at<uint32_t>(ws, P.off_boff), ws_at<float>(ws, P.off_ckpt),
                     ws_at<uint2>(ws, P.off_bq), P.ckpt_slots, ws_at<int32_t>(ws, P.off_flags),
                     P.vt, color, depth, last, dL_dcolor, dL_ddepth, target_rgb, target_depth,
                     fused, P.cfg.lambda_depth, ws_at<float>(ws, P.off_grad_pair));
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t fwd_launch(const Plan& P, void* ws, const float* cams, float* color, float* depth,
                      float* T_final, uint32_t* last, const float* target_rgb,
                      const float* target_depth, const uint32_t* order, int32_t* queue,
                      int grid, const TileSortArgs& sort, hipStream_t s) {
  const int B = P.cfg.lds_batch;
  const size_t lds = std::max((size_t)B * sizeof(Rec),
                              sort.cnt ? (size_t)kTileSortSmall * sizeof(uint64_t) : (size_t)0);
  if (P.cfg.flags & GS_SPLAT_BWD) {
    hipLaunchKernelGGL((k_render_fwd<TW, TH, true>), dim3(grid), dim3(kWave), lds, s,
                       rec_src(P, ws),
                       ws_at<uint32_t>(ws, P.off_ranges), cams, P.vt, B, color, depth, T_final,
                       last, ws_at<uint32_t>(ws, P.off_tile_last), target_rgb, target_depth,
                       ws_at<float>(ws, P.off_tile_loss), order, queue, P.cfg.chunk,
                       ws_at<uint32_t>(ws, P.off_boff), ws_at<float>(ws, P.off_ckpt), sort);
  } else {
    hipLaunchKernelGGL((k_render_fwd<TW, TH, false>), dim3(grid), dim3(kWave), lds, s,
                       rec_src(P, ws),
                       ws_at<uint32_t>(ws, P.off_ranges), cams, P.vt, B, color, depth, T_final,
                       last, ws_at<uint32_t>(ws, P.off_tile_last), target_rgb, target_depth,
                       ws_at<float>(ws, P.off_tile_loss), order, queue, P.cfg.chunk,
                       nullptr, nullptr, sort);
  }
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_launch(const Plan& P, void* ws, const float* cams, const float* color,
                      const float* depth, const float* T_final, const uint32_t* last,
                      const float* dL_dcolor, const float* dL_ddepth, const float* target_rgb,
                      const float* target_depth, int fused, const uint32_t* sorted_vals,
                      const uint32_t* order, int32_t* queue, int grid, hipStream_t s) {
  const int B = P.cfg.lds_batch;
  const size_t lds = (size_t)B * (sizeof(Rec) + sizeof(uint32_t));
  hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3(grid), dim3(kWave), lds, s,
                     rec_src(P, ws), sorted_vals,
                     ws_at<uint32_t>(ws, P.off_ranges), ws_at<uint32_t>(ws, P.off_tile_last), cams,
                     P.vt, B, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb,
                     target_depth, fused, P.cfg.lambda_depth,
                     ws_at<float>(ws, P.off_grad_pair), order, queue, P.cfg.chunk);
  return hipGetLastError();
}

template <typename K>
int occupancy(K kernel, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, kWave, lds) != hipSuccess || n < 1)
    n = 4;
  return n;
}

}  // namespace

// Resident single-wave workgroups per CU of the render kernel for this plan.
int render_blocks_per_cu(const Plan& P, bool bwd) {
  const int B = P.cfg.lds_batch;
  const size_t lf = (size_t)B * sizeof(Rec), lb = (size_t)B * (sizeof(Rec) + sizeof(uint32_t));
  const int tw = P.cfg.tile_w, th = P.cfg.tile_h;
  if (tw == 16 && th == 16) return bwd ? occupancy(k_render_bwd<16, 16>, lb) : occupancy(k_render_fwd<16, 16, false>, lf);
  if (tw == 16 && th == 8) return bwd ? occupancy(k_render_bwd<16, 8>, lb) : occupancy(k_render_fwd<16, 8, false>, lf);
  return bwd ? occupancy(k_render_bwd<8, 8>, lb) : occupancy(k_render_fwd<8, 8, false>, lf);
}

// Resident workgroups per CU of the splat-wise backward.
int splat_blocks_per_cu(const Plan& P) {
  const int tw = P.cfg.tile_w, th = P.cfg.tile_h;
  if (tw == 16 && th == 16) return occupancy(k_render_bwd_splat<16, 16>, 0);
  if (tw == 16 && th == 8) return occupancy(k_render_bwd_splat<16, 8>, 0);
  return occupancy(k_render_bwd_splat<8, 8>, 0);
}

// sort (optional, cnt non-null): the forward sorts each tile's short list
// itself (a whole iteration whose binning deferred those sorts).
hipError_t launch_render_fwd(const Plan& P, void* ws, const float* cams, float* color,
                             float* depth, float* T_final, uint32_t* last,
                             const float* target_rgb, const float* target_depth,
                             float* loss_per_view, const uint32_t* order, int32_t* queue,
                             int grid, hipStream_t s, const TileSortArgs& sort) {
  if (P.vt.total_tiles == 0) return hipSuccess;
  hipError_t e;
  const int tw = P.cfg.tile_w, th = P.cfg.tile_h;
  if (tw == 16 && th == 16)
    e = fwd_launch<16, 16>(P, ws, cams, color, depth, T_final, last, target_rgb, target_depth, order, queue, grid, sort, s);
  else if (tw == 16 && th == 8)
    e = fwd_launch<16, 8>(P, ws, cams, color, depth, T_final, last, target_rgb, target_depth, order, queue, grid, sort, s);
  else
    e = fwd_launch<8, 8>(P, ws, cams, color, depth, T_final, last, target_rgb, target_depth, order, queue, grid, sort, s);
  if (e != hipSuccess) return e;
  if (target_rgb && loss_per_view) {
    hipLaunchKernelGGL(k_loss_reduce, dim3(P.vt.n_views), dim3(kLossThreads), 0, s,
                       ws_at<float>(ws, P.off_tile_loss), P.vt, P.cfg.lambda_depth,
                       target_depth ? 1 : 0, loss_per_view);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_render_bwd(const Plan& P, void* ws, const float* cams, const float* color,
                             const float* depth, const float* T_final, const uint32_t* last,
                             const float* dL_dcolor, const float* dL_ddepth,
                             const float* target_rgb, const float* target_depth, int fused,
                             const uint32_t* sorted_vals, const uint32_t* order, int32_t* queue,
                             int grid, hipStream_t s) {
  if (P.vt.total_tiles == 0) return hipSuccess;
  const int tw = P.cfg.tile_w, th = P.cfg.tile_h;
  if (P.cfg.flags & GS_SPLAT_BWD) {
    if (tw == 16 && th == 16)
      return bwd_splat_launch<16, 16>(P, ws, cams, color, depth, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, grid, s);
    if (tw == 16 && th == 8)
      return bwd_splat_launch<16, 8>(P, ws, cams, color, depth, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, grid, s);
    return bwd_splat_launch<8, 8>(P, ws, cams, color, depth, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, grid, s);
  }
  if (tw == 16 && th == 16)
    return bwd_launch<16, 16>(P, ws, cams, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, order, queue, grid, s);
  if (tw == 16 && th == 8)
    return bwd_launch<16, 8>(P, ws, cams, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, order, queue, grid, s);
  return bwd_launch<8, 8>(P, ws, cams, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, order, queue, grid, s);
}

}  // namespace gs

// a3-a5: per-tile compositing (Eq. (1)) and its pixel-wise backward
// (Eqs. (2)-(4)), one workgroup per tile, one lane per pixel.
//
// Forward: records of the tile's depth-sorted list are staged in LDS in
// batches; every lane walks the batch front to back.  A wavefront leaves the
// batch loop as soon as the ballot of its unfinished lanes is empty, and the
// workgroup stops staging batches once no lane of any wavefront is left.
//
// Backward: back to front from each tile's last used position.  Each lane
// recomputes alpha with the same code as the forward (so every skip decision
// is the forward's), undoes the transmittance by division starting from
// T_final, and keeps the running sums of what lies behind.  The ten per-pair
// partial gradients are summed across the wavefront (skipped when no lane
// contributes), the wavefront sums are combined in LDS in a fixed order, and
// each (tile, Gaussian) pair writes its own slot: no atomics, and the result
// is deterministic.
#include "gs_internal.h"

namespace gs {
namespace {

constexpr double kLog2e = 1.4426950408889634;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;

// alpha of record r at sample point (sx, sy).  Returns false when the
// Gaussian is skipped (positive exponent or alpha < 1/255).  The quadratic
// form is evaluated in FP64; the exponential in FP32.
__device__ __forceinline__ bool eval_alpha(const Rec& r, double sx, double sy, double& dx,
                                           double& dy, float& G, float& oG, float& a) {
  dx = r.mx - sx;
  dy = r.my - sy;
  const double pw = fma(dx, fma(r.ca, dx, r.cb * dy), (r.cc * dy) * dy);
  if (pw > 0.0) return false;
  G = __builtin_amdgcn_exp2f((float)(pw * kLog2e));
  oG = r.o * G;
  a = fminf(kAlphaMax, oG);
  return a >= kAlphaMin;
}

__device__ __forceinline__ int find_view(const ViewTable& vt, int gtile) {
  int v = 0;
  while (v + 1 < vt.n_views && gtile >= vt.v[v + 1].tile_off) ++v;
  return v;
}

__device__ __forceinline__ void stage_records(Rec* srec, const Rec* __restrict__ rec,
                                              const uint32_t* __restrict__ sorted_rec,
                                              uint32_t first, int count, int nthreads) {
  for (int k = threadIdx.x; k < count; k += nthreads) {
    const float4* src = reinterpret_cast<const float4*>(rec + sorted_rec[first + k]);
    float4* dst = reinterpret_cast<float4*>(srec + k);
    const float4 a0 = src[0], a1 = src[1], a2 = src[2], a3 = src[3];
    dst[0] = a0; dst[1] = a1; dst[2] = a2; dst[3] = a3;
  }
}

// ------------------------------------------------------------------ forward
template <int TW, int TH>
__device__ __forceinline__ void fwd_tile(int gtile, const Rec* __restrict__ rec,
                                         const uint32_t* __restrict__ sorted_rec,
                                         const uint32_t* __restrict__ ranges,
                                         const float* __restrict__ cams, const ViewTable& vt,
                                         int B, float* __restrict__ color,
                                         float* __restrict__ depth, float* __restrict__ T_final,
                                         uint32_t* __restrict__ last,
                                         uint32_t* __restrict__ tile_last,
                                         const float* __restrict__ target_rgb,
                                         const float* __restrict__ target_depth,
                                         float* __restrict__ tile_loss, Rec* srec,
                                         uint32_t* sred, float* sloss) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / kWave;
  const int v = find_view(vt, gtile);
  const ViewInfo vi = vt.v[v];
  const int lt = gtile - vi.tile_off;
  const int tx0 = (lt % vi.tiles_x) * TW, ty0 = (lt / vi.tiles_x) * TH;
  const int t = threadIdx.x;
  const int px = tx0 + t % TW, py = ty0 + t / TW;
  const bool inside = (px < vi.W) && (py < vi.H);
  const double sx = px + 0.5, sy = py + 0.5;
  const uint32_t s = ranges[2 * (int64_t)gtile], e = ranges[2 * (int64_t)gtile + 1];

  float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, D = 0.0f;
  uint32_t lastpos = 0;
  bool done = !inside;
  for (uint32_t b = s; b < e; b += (uint32_t)B) {
    const int nb = (int)min((uint32_t)B, e - b);
    if (__syncthreads_count(done ? 0 : 1) == 0) break;
    stage_records(srec, rec, sorted_rec, b, nb, NT);
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      if (!done) {
        const Rec& r = srec[j];
        double dx, dy;
        float G, oG, a;
        if (eval_alpha(r, sx, sy, dx, dy, G, oG, a)) {
          const float Tn = T * (1.0f - a);
          if (Tn < kTMin) {
            done = true;
          } else {
            const float w = a * T;
            c0 = fmaf(r.r, w, c0);
            c1 = fmaf(r.g, w, c1);
            c2 = fmaf(r.b, w, c2);
            D = fmaf(r.z, w, D);
            T = Tn;
            lastpos = b - s + (uint32_t)j + 1u;
          }
        }
      }
      if (ballot64(!done) == 0) break;
    }
  }
  const float* cam = cams + (int64_t)v * GS_CAMERA_FLOATS;
  float lrgb = 0.0f, ld = 0.0f;
  if (inside) {
    const int64_t npx = (int64_t)vi.W * vi.H;
    const int64_t pl = (int64_t)py * vi.W + px;
    const int64_t pix = (int64_t)vi.pix_off + pl;
    const int64_t cbase = 3 * (int64_t)vi.pix_off + pl;
    const float o0 = fmaf(T, cam[17], c0), o1 = fmaf(T, cam[18], c1), o2 = fmaf(T, cam[19], c2);
    color[cbase] = o0;
    color[cbase + npx] = o1;
    color[cbase + 2 * npx] = o2;
    depth[pix] = D;
    T_final[pix] = T;
    last[pix] = lastpos;
    if (target_rgb) {
      lrgb = fabsf(o0 - target_rgb[cbase]) + fabsf(o1 - target_rgb[cbase + npx]) +
             fabsf(o2 - target_rgb[cbase + 2 * npx]);
      if (target_depth) ld = fabsf(D - target_depth[pix]);
    }
  }
  // per-tile maximum of `last` (where the backward starts) and loss sums
  const uint32_t m = wave_max(lastpos);
  float sl0 = 0.0f, sl1 = 0.0f;
  if (target_rgb) {
    sl0 = wave_sum(lrgb);
    sl1 = wave_sum(ld);
  }
  const int w = t / kWave;
  if (lane_id() == 0) {
    sred[w] = m;
    sloss[2 * w] = sl0;
    sloss[2 * w + 1] = sl1;
  }
  __syncthreads();
  if (t == 0) {
    uint32_t mm = 0;
    float a0 = 0.0f, a1 = 0.0f;
    for (int k = 0; k < NW; ++k) {
      mm = max(mm, sred[k]);
      a0 += sloss[2 * k];
      a1 += sloss[2 * k + 1];
    }
    tile_last[gtile] = mm;
    if (target_rgb) {
      tile_loss[2 * (int64_t)gtile] = a0;
      tile_loss[2 * (int64_t)gtile + 1] = a1;
    }
  }
  __syncthreads();
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) k_render_fwd(
    const Rec* __restrict__ rec, const uint32_t* __restrict__ sorted_rec,
    const uint32_t* __restrict__ ranges, const float* __restrict__ cams, ViewTable vt, int B,
    float* __restrict__ color, float* __restrict__ depth, float* __restrict__ T_final,
    uint32_t* __restrict__ last, uint32_t* __restrict__ tile_last,
    const float* __restrict__ target_rgb, const float* __restrict__ target_depth,
    float* __restrict__ tile_loss, const uint32_t* __restrict__ order,
    int32_t* __restrict__ queue, int chunk) {
  extern __shared__ __align__(16) unsigned char smem[];
  Rec* srec = reinterpret_cast<Rec*>(smem);
  __shared__ uint32_t sred[(TW * TH) / kWave];
  __shared__ float sloss[2 * (TW * TH) / kWave];
  __shared__ int swork;
  if (queue == nullptr) {
    const int g = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    fwd_tile<TW, TH>(g, rec, sorted_rec, ranges, cams, vt, B, color, depth, T_final, last,
                     tile_last, target_rgb, target_depth, tile_loss, srec, sred, sloss);
    return;
  }
  // persistent: pull chunks of `chunk` tiles until the queue is drained
  const int n_items = (vt.total_tiles + chunk - 1) / chunk;
  for (;;) {
    if (threadIdx.x == 0) swork = atomicAdd(queue, 1);
    __syncthreads();
    const int item = swork;
    __syncthreads();
    if (item >= n_items) break;
    const int first = item * chunk;
    const int lastt = min(vt.total_tiles, first + chunk);
    for (int k = first; k < lastt; ++k) {
      const int g = order ? (int)order[k] : k;
      fwd_tile<TW, TH>(g, rec, sorted_rec, ranges, cams, vt, B, color, depth, T_final, last,
                       tile_last, target_rgb, target_depth, tile_loss, srec, sred, sloss);
    }
  }
}

// Per-view L1 loss from the per-tile sums, in a fixed order.
__global__ void __launch_bounds__(256) k_loss_reduce(const float* __restrict__ tile_loss,
                                                     ViewTable vt, float lambda_depth,
                                                     int has_depth, float* __restrict__ loss) {
  const int v = blockIdx.x;
  const ViewInfo vi = vt.v[v];
  const int nt = vi.tiles_x * vi.tiles_y;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nt; k += 256) {
    a += tile_loss[2 * (int64_t)(vi.tile_off + k)];
    b += tile_loss[2 * (int64_t)(vi.tile_off + k) + 1];
  }
  __shared__ double sa[256 / kWave], sb[256 / kWave];
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane_id() == 0) {
    sa[threadIdx.x / kWave] = a;
    sb[threadIdx.x / kWave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int k = 0; k < 256 / kWave; ++k) {
      ta += sa[k];
      tb += sb[k];
    }
    const double npx = (double)vi.W * vi.H;
    loss[v] = (float)(ta / (3.0 * npx) + (has_depth ? lambda_depth * tb / npx : 0.0));
  }
}

// ------------------------------------------------------------------ backward
template <int TW, int TH>
__device__ __forceinline__ void bwd_tile(
    int gtile, const Rec* __restrict__ rec, const uint32_t* __restrict__ sorted_rec,
    const uint32_t* __restrict__ sorted_vals, const uint32_t* __restrict__ ranges,
    const uint32_t* __restrict__ tile_last, const float* __restrict__ cams, const ViewTable& vt,
    int B, const float* __restrict__ color, const float* __restrict__ depth,
    const float* __restrict__ T_final, const uint32_t* __restrict__ last,
    const float* __restrict__ dL_dcolor, const float* __restrict__ dL_ddepth,
    const float* __restrict__ target_rgb, const float* __restrict__ target_depth, int fused,
    float lambda_depth, float* __restrict__ grad_pair, Rec* srec, float* spart) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / kWave;
  const int v = find_view(vt, gtile);
  const ViewInfo vi = vt.v[v];
  const int lt = gtile - vi.tile_off;
  const int tx0 = (lt % vi.tiles_x) * TW, ty0 = (lt / vi.tiles_x) * TH;
  const int t = threadIdx.x;
  const int w = t / kWave;
  const int lane = lane_id();
  const int px = tx0 + t % TW, py = ty0 + t / TW;
  const bool inside = (px < vi.W) && (py < vi.H);
  const double sx = px + 0.5, sy = py + 0.5;
  const uint32_t s = ranges[2 * (int64_t)gtile], e = ranges[2 * (int64_t)gtile + 1];
  const uint32_t tl = tile_last[gtile];
  const float* cam = cams + (int64_t)v * GS_CAMERA_FLOATS;

  // pairs beyond the last used position get zero gradients
  for (uint32_t k = tl + (uint32_t)t; k < e - s; k += NT) {
    float4* gp = reinterpret_cast<float4*>(grad_pair + (int64_t)sorted_vals[s + k] * kPairGrad);
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    gp[0] = z; gp[1] = z; gp[2] = z;
  }

  float T = 1.0f, gC0 = 0.0f, gC1 = 0.0f, gC2 = 0.0f, gD = 0.0f;
  uint32_t L = 0;
  if (inside) {
    const int64_t npx = (int64_t)vi.W * vi.H;
    const int64_t pl = (int64_t)py * vi.W + px;
    const int64_t pix = (int64_t)vi.pix_off + pl;
    const int64_t cbase = 3 * (int64_t)vi.pix_off + pl;
    T = T_final[pix];
    L = last[pix];
    if (fused) {
      const float inv3 = 1.0f / (3.0f * (float)npx);
      const float c0 = color[cbase], c1 = color[cbase + npx], c2 = color[cbase + 2 * npx];
      const float d0 = c0 - target_rgb[cbase], d1 = c1 - target_rgb[cbase + npx],
                  d2 = c2 - target_rgb[cbase + 2 * npx];
      gC0 = d0 > 0.0f ? inv3 : (d0 < 0.0f ? -inv3 : 0.0f);
      gC1 = d1 > 0.0f ? inv3 : (d1 < 0.0f ? -inv3 : 0.0f);
      gC2 = d2 > 0.0f ? inv3 : (d2 < 0.0f ? -inv3 : 0.0f);
      if (target_depth) {
        const float dd = depth[pix] - target_depth[pix];
        const float sc = lambda_depth / (float)npx;
        gD = dd > 0.0f ? sc : (dd < 0.0f ? -sc : 0.0f);
      }
    } else {
      gC0 = dL_dcolor[cbase];
      gC1 = dL_dcolor[cbase + npx];
      gC2 = dL_dcolor[cbase + 2 * npx];
      gD = dL_ddepth ? dL_ddepth[pix] : 0.0f;
    }
  }
  // behind-sums: background seen through T_final, nothing behind in depth
  float Sc0 = T * cam[17], Sc1 = T * cam[18], Sc2 = T * cam[19], Sd = 0.0f;

  for (int bend = (int)tl; bend > 0; bend -= B) {
    const int bstart = max(0, bend - B);
    const int nb = bend - bstart;
    __syncthreads();
    stage_records(srec, rec, sorted_rec, s + (uint32_t)bstart, nb, NT);
    for (int k = t; k < NW * nb * 10; k += NT) spart[k] = 0.0f;
    __syncthreads();
    for (int j = nb - 1; j >= 0; --j) {
      const uint32_t pos = (uint32_t)(bstart + j);
      float g[10];
#pragma unroll
      for (int f = 0; f < 10; ++f) g[f] = 0.0f;
      bool contrib = false;
      if (pos < L) {
        const Rec& r = srec[j];
        double dx, dy;
        float G, oG, a;
        if (eval_alpha(r, sx, sy, dx, dy, G, oG, a)) {
          contrib = true;
          const float inv_om = __builtin_amdgcn_rcpf(1.0f - a);
          const float Tk = T * inv_om;
          const float wgt = a * Tk;
          g[0] = wgt * gC0;
          g[1] = wgt * gC1;
          g[2] = wgt * gC2;
          g[3] = wgt * gD;
          const float front = gC0 * r.r + gC1 * r.g + gC2 * r.b + gD * r.z;
          const float behind = gC0 * Sc0 + gC1 * Sc1 + gC2 * Sc2 + gD * Sd;
          const float g_alpha = Tk * front - behind * inv_om;
          Sc0 = fmaf(r.r, wgt, Sc0);
          Sc1 = fmaf(r.g, wgt, Sc1);
          Sc2 = fmaf(r.b, wgt, Sc2);
          Sd = fmaf(r.z, wgt, Sd);
          T = Tk;
          if (oG <= kAlphaMax) {
            const float gpow = a * g_alpha;
            const float fx = (float)dx, fy = (float)dy;
            const float ca = (float)(-2.0 * r.ca), cb = (float)(-r.cb), cc = (float)(-2.0 * r.cc);
            g[4] = G * g_alpha;
            g[5] = -0.5f * gpow * fx * fx;
            g[6] = -gpow * fx * fy;
            g[7] = -0.5f * gpow * fy * fy;
            g[8] = -gpow * (ca * fx + cb * fy);
            g[9] = -gpow * (cb * fx + cc * fy);
          }
        }
      }
      if (ballot64(contrib) != 0) {
#pragma unroll
        for (int f = 0; f < 10; ++f) g[f] = wave_sum(g[f]);
        if (lane == 0) {
#pragma unroll
          for (int f = 0; f < 10; ++f) spart[(w * nb + j) * 10 + f] = g[f];
        }
      }
    }
    __syncthreads();
    // combine wavefronts in a fixed order; one slot per (tile, Gaussian)
    for (int k = t; k < nb; k += NT) {
      float acc[10];
#pragma unroll
      for (int f = 0; f < 10; ++f) acc[f] = spart[k * 10 + f];
      for (int ww = 1; ww < NW; ++ww)
#pragma unroll
        for (int f = 0; f < 10; ++f) acc[f] += spart[(ww * nb + k) * 10 + f];
      float4* gp =
          reinterpret_cast<float4*>(grad_pair + (int64_t)sorted_vals[s + bstart + k] * kPairGrad);
      gp[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      gp[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
      gp[2] = make_float4(acc[8], acc[9], 0.0f, 0.0f);
    }
  }
  __syncthreads();
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW* TH) k_render_bwd(
    const Rec* __restrict__ rec, const uint32_t* __restrict__ sorted_rec,
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
  float* spart = reinterpret_cast<float*>(smem + (size_t)B * sizeof(Rec));
  __shared__ int swork;
  if (queue == nullptr) {
    const int g = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    bwd_tile<TW, TH>(g, rec, sorted_rec, sorted_vals, ranges, tile_last, cams, vt, B, color, depth,
                     T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused,
                     lambda_depth, grad_pair, srec, spart);
    return;
  }
  const int n_items = (vt.total_tiles + chunk - 1) / chunk;
  for (;;) {
    if (threadIdx.x == 0) swork = atomicAdd(queue, 1);
    __syncthreads();
    const int item = swork;
    __syncthreads();
    if (item >= n_items) break;
    const int first = item * chunk;
    const int lastt = min(vt.total_tiles, first + chunk);
    for (int k = first; k < lastt; ++k) {
      const int g = order ? (int)order[k] : k;
      bwd_tile<TW, TH>(g, rec, sorted_rec, sorted_vals, ranges, tile_last, cams, vt, B, color,
                       depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth,
                       fused, lambda_depth, grad_pair, srec, spart);
    }
  }
}

template <int TW, int TH>
hipError_t fwd_launch(const Plan& P, void* ws, const float* cams, float* color, float* depth,
                      float* T_final, uint32_t* last, const float* target_rgb,
                      const float* target_depth, const uint32_t* order, int32_t* queue,
                      int grid, hipStream_t s) {
  const int B = P.cfg.lds_batch;
  const size_t lds = (size_t)B * sizeof(Rec);
  hipLaunchKernelGGL((k_render_fwd<TW, TH>), dim3(grid), dim3(TW * TH), lds, s,
                     ws_at<Rec>(ws, P.off_rec), ws_at<uint32_t>(ws, P.off_sorted_rec),
                     ws_at<uint32_t>(ws, P.off_ranges), cams, P.vt, B, color, depth, T_final,
                     last, ws_at<uint32_t>(ws, P.off_tile_last), target_rgb, target_depth,
                     ws_at<float>(ws, P.off_tile_loss), order, queue, P.cfg.chunk);
  return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_launch(const Plan& P, void* ws, const float* cams, const float* color,
                      const float* depth, const float* T_final, const uint32_t* last,
                      const float* dL_dcolor, const float* dL_ddepth, const float* target_rgb,
                      const float* target_depth, int fused, const uint32_t* sorted_vals,
                      const uint32_t* order, int32_t* queue, int grid, hipStream_t s) {
  constexpr int NW = TW * TH / kWave;
  const int B = P.cfg.lds_batch;
  const size_t lds = (size_t)B * sizeof(Rec) + (size_t)NW * B * 10 * sizeof(float);
  hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3(grid), dim3(TW * TH), lds, s,
                     ws_at<Rec>(ws, P.off_rec), ws_at<uint32_t>(ws, P.off_sorted_rec), sorted_vals,
                     ws_at<uint32_t>(ws, P.off_ranges), ws_at<uint32_t>(ws, P.off_tile_last), cams,
                     P.vt, B, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb,
                     target_depth, fused, P.cfg.lambda_depth,
                     ws_at<float>(ws, P.off_grad_pair), order, queue, P.cfg.chunk);
  return hipGetLastError();
}

}  // namespace

size_t render_bwd_lds_bytes(const Plan& P) {
  const int NW = P.cfg.tile_w * P.cfg.tile_h / kWave;
  return (size_t)P.cfg.lds_batch * sizeof(Rec) + (size_t)NW * P.cfg.lds_batch * 10 * sizeof(float);
}

hipError_t launch_render_fwd(const Plan& P, void* ws, const float* cams, float* color,
                             float* depth, float* T_final, uint32_t* last,
                             const float* target_rgb, const float* target_depth,
                             float* loss_per_view, const uint32_t* order, int32_t* queue,
                             int grid, hipStream_t s) {
  if (P.vt.total_tiles == 0) return hipSuccess;
  hipError_t e;
  const int tw = P.cfg.tile_w, th = P.cfg.tile_h;
  if (tw == 16 && th == 16)
    e = fwd_launch<16, 16>(P, ws, cams, color, depth, T_final, last, target_rgb, target_depth, order, queue, grid, s);
  else if (tw == 16 && th == 8)
    e = fwd_launch<16, 8>(P, ws, cams, color, depth, T_final, last, target_rgb, target_depth, order, queue, grid, s);
  else
    e = fwd_launch<8, 8>(P, ws, cams, color, depth, T_final, last, target_rgb, target_depth, order, queue, grid, s);
  if (e != hipSuccess) return e;
  if (target_rgb && loss_per_view) {
    hipLaunchKernelGGL(k_loss_reduce, dim3(P.vt.n_views), dim3(256), 0, s,
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
  if (tw == 16 && th == 16)
    return bwd_launch<16, 16>(P, ws, cams, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, order, queue, grid, s);
  if (tw == 16 && th == 8)
    return bwd_launch<16, 8>(P, ws, cams, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, order, queue, grid, s);
  return bwd_launch<8, 8>(P, ws, cams, color, depth, T_final, last, dL_dcolor, dL_ddepth, target_rgb, target_depth, fused, sorted_vals, order, queue, grid, s);
}

}  // namespace gs

// Rendered loss of Eq. (9) with a depth term:
//   L = (1 - ls) mean|C - C*| + ls (1 - SSIM(C, C*)) + ld mean|D - D*|
// and its image gradients dL/dC, dL/dD, which then drive the raster
// backward as explicit upstream gradients.  SSIM follows the 3DGS pipeline
// the paper retains (Sec. IV-A): per channel, 11x11 Gaussian window with
// sigma 1.5, zero padding, C1 = 0.01^2, C2 = 0.03^2.
//
// Stencil work on 16x16 output tiles: the 26x26 halo of the image (and the
// target) is staged in LDS, filtered along rows then columns.  Pass 1 forms
// the five windowed moments, the SSIM value and its derivatives with respect
// to the moments of C (three maps); pass 2 filters those maps with the
// (symmetric) window -- the adjoint of the forward filtering -- and
// assembles dL/dC.  Per-tile sums are reduced per view in a fixed order.
#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kT = 16;            // output tile edge
constexpr int kR = 5;             // window radius
constexpr int kH = kT + 2 * kR;   // halo edge, 26
constexpr float kC1 = 1e-4f;      // 0.01^2
constexpr float kC2 = 9e-4f;      // 0.03^2

__constant__ float c_win[11] = {
    0.0010284048259f, 0.0075987582919f, 0.0360007721186f, 0.1093606895208f,
    0.2130055377627f, 0.2660117248603f, 0.2130055377627f, 0.1093606895208f,
    0.0360007721186f, 0.0075987582919f, 0.0010284048259f};

struct SsimView {
  int32_t W, H, tiles_x, tile_off, pix_off;
};
struct SsimTable {
  int32_t n_views, total_tiles;
  SsimView v[kMaxViews];
};

__device__ __forceinline__ int ssim_view(const SsimTable& t, int tile) {
  int v = 0;
  while (v + 1 < t.n_views && tile >= t.v[v + 1].tile_off) ++v;
  return v;
}

// Pass 1: grid (tiles over all views, 3 channels), 256 threads.
__global__ void __launch_bounds__(256) k_ssim_fwd(const float* __restrict__ color,
                                                  const float* __restrict__ target,
                                                  SsimTable tb, float* __restrict__ dmaps,
                                                  float* __restrict__ part) {
  __shared__ float sx[kH][kH + 1], sy[kH][kH + 1];
  __shared__ float hm[5][kH][kT + 1];
  __shared__ float red[2][256 / kWave];
  const int tile = blockIdx.x, ch = blockIdx.y;
  const int v = ssim_view(tb, tile);
  const SsimView vi = tb.v[v];
  const int lt = tile - vi.tile_off;
  const int x0 = (lt % vi.tiles_x) * kT - kR, y0 = (lt / vi.tiles_x) * kT - kR;
  const int64_t npx = (int64_t)vi.W * vi.H;
  const float* X = color + 3 * (int64_t)vi.pix_off + ch * npx;
  const float* Y = target + 3 * (int64_t)vi.pix_off + ch * npx;
  for (int k = threadIdx.x; k < kH * kH; k += 256) {
    const int r = k / kH, c = k % kH, gx = x0 + c, gy = y0 + r;
    const bool in = gx >= 0 && gy >= 0 && gx < vi.W && gy < vi.H;
    sx[r][c] = in ? X[(int64_t)gy * vi.W + gx] : 0.0f;
    sy[r][c] = in ? Y[(int64_t)gy * vi.W + gx] : 0.0f;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kH * kT; k += 256) {
    const int r = k / kT, c = k % kT;
    float a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
#pragma unroll
    for (int j = 0; j < 11; ++j) {
      const float w = c_win[j], x = sx[r][c + j], y = sy[r][c + j];
      a0 = fmaf(w, x, a0);
      a1 = fmaf(w, y, a1);
      a2 = fmaf(w, x * x, a2);
      a3 = fmaf(w, y * y, a3);
      a4 = fmaf(w, x * y, a4);
    }
    hm[0][r][c] = a0; hm[1][r][c] = a1; hm[2][r][c] = a2; hm[3][r][c] = a3; hm[4][r][c] = a4;
  }
  __syncthreads();
  const int c = threadIdx.x % kT, r = threadIdx.x / kT;
  float m[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < 11; ++j) {
    const float w = c_win[j];
#pragma unroll
    for (int q = 0; q < 5; ++q) m[q] = fmaf(w, hm[q][r + j][c], m[q]);
  }
  const int gx = x0 + kR + c, gy = y0 + kR + r;
  const bool in = gx < vi.W && gy < vi.H;
  float s_val = 0.0f, l1 = 0.0f;
  if (in) {
    const float m1 = m[0], my = m[1], m2 = m[2], myy = m[3], m3 = m[4];
    const float A1 = 2.0f * m1 * my + kC1;
    const float A2 = 2.0f * (m3 - m1 * my) + kC2;
    const float B1 = m1 * m1 + my * my + kC1;
    const float B2 = (m2 - m1 * m1) + (myy - my * my) + kC2;
    const float S = (A1 * A2) / (B1 * B2);
    const float d1 = S * (2.0f * my / A1 - 2.0f * my / A2 - 2.0f * m1 / B1 + 2.0f * m1 / B2);
    const float d2 = -S / B2;
    const float d3 = 2.0f * S / A2;
    const int64_t p = 3 * ((int64_t)vi.pix_off * 3 + ch * npx + (int64_t)gy * vi.W + gx);
    dmaps[p] = d1;
    dmaps[p + 1] = d2;
    dmaps[p + 2] = d3;
    s_val = S;
    l1 = fabsf(sx[r + kR][c + kR] - sy[r + kR][c + kR]);
  }
  s_val = wave_sum(s_val);
  l1 = wave_sum(l1);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = s_val;
    red[1][threadIdx.x / kWave] = l1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0, b = 0;
    for (int k = 0; k < 256 / kWave; ++k) {
      a += red[0][k];
      b += red[1][k];
    }
    part[4 * ((int64_t)tile * 3 + ch)] = a;
    part[4 * ((int64_t)tile * 3 + ch) + 1] = b;
  }
}

// Pass 2: adjoint filtering of the derivative maps, dL/dC and dL/dD.
__global__ void __launch_bounds__(256) k_ssim_bwd(
    const float* __restrict__ color, const float* __restrict__ target,
    const float* __restrict__ depth, const float* __restrict__ target_depth, SsimTable tb,
    const float* __restrict__ dmaps, float lambda_ssim, float lambda_depth,
    float* __restrict__ dL_dcolor, float* __restrict__ dL_ddepth, float* __restrict__ part) {
  __shared__ float sd[3][kH][kH + 1];
  __shared__ float hm[3][kH][kT + 1];
  __shared__ float red[256 / kWave];
  const int tile = blockIdx.x, ch = blockIdx.y;
  const int v = ssim_view(tb, tile);
  const SsimView vi = tb.v[v];
  const int lt = tile - vi.tile_off;
  const int x0 = (lt % vi.tiles_x) * kT - kR, y0 = (lt / vi.tiles_x) * kT - kR;
  const int64_t npx = (int64_t)vi.W * vi.H;
  const int64_t cbase = 3 * (int64_t)vi.pix_off + ch * npx;
  for (int k = threadIdx.x; k < kH * kH; k += 256) {
    const int r = k / kH, c = k % kH, gx = x0 + c, gy = y0 + r;
    const bool in = gx >= 0 && gy >= 0 && gx < vi.W && gy < vi.H;
    const int64_t p = 3 * (cbase + (int64_t)gy * vi.W + gx);
    sd[0][r][c] = in ? dmaps[p] : 0.0f;
    sd[1][r][c] = in ? dmaps[p + 1] : 0.0f;
    sd[2][r][c] = in ? dmaps[p + 2] : 0.0f;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kH * kT; k += 256) {
    const int r = k / kT, c = k % kT;
    float a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int j = 0; j < 11; ++j) {
      const float w = c_win[j];
      a0 = fmaf(w, sd[0][r][c + j], a0);
      a1 = fmaf(w, sd[1][r][c + j], a1);
      a2 = fmaf(w, sd[2][r][c + j], a2);
    }
    hm[0][r][c] = a0; hm[1][r][c] = a1; hm[2][r][c] = a2;
  }
  __syncthreads();
  const int c = threadIdx.x % kT, r = threadIdx.x / kT;
  float g1 = 0, g2 = 0, g3 = 0;
#pragma unroll
  for (int j = 0; j < 11; ++j) {
    const float w = c_win[j];
    g1 = fmaf(w, hm[0][r + j][c], g1);
    g2 = fmaf(w, hm[1][r + j][c], g2);
    g3 = fmaf(w, hm[2][r + j][c], g3);
  }
  const int gx = x0 + kR + c, gy = y0 + kR + r;
  const bool in = gx < vi.W && gy < vi.H;
  float ld = 0.0f;
  if (in) {
    const int64_t p = cbase + (int64_t)gy * vi.W + gx;
    const float x = color[p], y = target[p];
    const float inv_n = 1.0f / (3.0f * (float)npx);
    const float dssim = (g1 + 2.0f * x * g2 + y * g3) * inv_n;
    const float dx = x - y;
    const float sgn = dx > 0.0f ? 1.0f : (dx < 0.0f ? -1.0f : 0.0f);
    dL_dcolor[p] = (1.0f - lambda_ssim) * sgn * inv_n - lambda_ssim * dssim;
    if (ch == 0) {
      const int64_t q = (int64_t)vi.pix_off + (int64_t)gy * vi.W + gx;
      float gd = 0.0f;
      if (target_depth) {
        const float dd = depth[q] - target_depth[q];
        gd = dd > 0.0f ? lambda_depth / (float)npx : (dd < 0.0f ? -lambda_depth / (float)npx : 0.0f);
        ld = fabsf(dd);
      }
      dL_ddepth[q] = gd;
    }
  }
  if (ch == 0) {
    ld = wave_sum(ld);
    if (lane_id() == 0) red[threadIdx.x / kWave] = ld;
    __syncthreads();
    if (threadIdx.x == 0) {
      float a = 0;
      for (int k = 0; k < 256 / kWave; ++k) a += red[k];
      part[4 * ((int64_t)tile * 3) + 2] = a;
    }
  }
}

// Per-view loss from the per-tile sums, fixed order.
__global__ void __launch_bounds__(256) k_ssim_loss(const float* __restrict__ part, SsimTable tb,
                                                   float lambda_ssim, float lambda_depth,
                                                   int has_depth, float* __restrict__ loss) {
  const int v = blockIdx.x;
  const SsimView vi = tb.v[v];
  const int nt = (v + 1 < tb.n_views ? tb.v[v + 1].tile_off : tb.total_tiles) - vi.tile_off;
  double s = 0, l1 = 0, ld = 0;
  for (int k = threadIdx.x; k < nt; k += 256) {
    const int64_t t = vi.tile_off + k;
    for (int ch = 0; ch < 3; ++ch) {
      s += part[4 * (t * 3 + ch)];
      l1 += part[4 * (t * 3 + ch) + 1];
    }
    ld += part[4 * (t * 3) + 2];
  }
  __shared__ double red[3][256 / kWave];
  s = wave_sum(s);
  l1 = wave_sum(l1);
  ld = wave_sum(ld);
  if (lane_id() == 0) {
    red[0][threadIdx.x / kWave] = s;
    red[1][threadIdx.x / kWave] = l1;
    red[2][threadIdx.x / kWave] = ld;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0;
    for (int k = 0; k < 256 / kWave; ++k) {
      a += red[0][k];
      b += red[1][k];
      c += red[2][k];
    }
    const double n3 = 3.0 * (double)vi.W * vi.H;
    double L = (1.0 - lambda_ssim) * b / n3 + lambda_ssim * (1.0 - a / n3);
    if (has_depth) L += lambda_depth * c / ((double)vi.W * vi.H);
    loss[v] = (float)L;
  }
}

}  // namespace

int64_t ssim_tiles(const Plan& P) {
  int64_t t = 0;
  for (int v = 0; v < P.vt.n_views; ++v)
    t += (int64_t)((P.vt.v[v].W + kT - 1) / kT) * ((P.vt.v[v].H + kT - 1) / kT);
  return t;
}

hipError_t launch_render_loss(const Plan& P, void* ws, const float* color, const float* depth,
                              const float* target_rgb, const float* target_depth,
                              double lambda_ssim, float* dL_dcolor, float* dL_ddepth,
                              float* loss_per_view, hipStream_t s) {
  SsimTable tb{};
  tb.n_views = P.vt.n_views;
  int32_t t = 0;
  for (int v = 0; v < P.vt.n_views; ++v) {
    const ViewInfo& vi = P.vt.v[v];
    SsimView& sv = tb.v[v];
    sv.W = vi.W;
    sv.H = vi.H;
    sv.tiles_x = (vi.W + kT - 1) / kT;
    sv.tile_off = t;
    sv.pix_off = vi.pix_off;
    t += sv.tiles_x * ((vi.H + kT - 1) / kT);
  }
  tb.total_tiles = t;
  if (t == 0) return hipSuccess;
  float* dmaps = ws_at<float>(ws, P.off_ssim_maps);
  float* part = ws_at<float>(ws, P.off_ssim_part);
  hipLaunchKernelGGL(k_ssim_fwd, dim3(t, 3), dim3(256), 0, s, color, target_rgb, tb, dmaps, part);
  hipLaunchKernelGGL(k_ssim_bwd, dim3(t, 3), dim3(256), 0, s, color, target_rgb, depth,
                     target_depth, tb, dmaps, (float)lambda_ssim, P.cfg.lambda_depth, dL_dcolor,
                     dL_ddepth, part);
  if (loss_per_view)
    hipLaunchKernelGGL(k_ssim_loss, dim3(P.vt.n_views), dim3(256), 0, s, part, tb,
                       (float)lambda_ssim, P.cfg.lambda_depth, target_depth ? 1 : 0,
                       loss_per_view);
  return hipGetLastError();
}

}  // namespace gs

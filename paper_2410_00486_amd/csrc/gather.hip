// Keyframe pool -> batch slots: the first launch of a scheduled iteration
// copies each selected keyframe's camera record and target images into its
// batch slot, so that a captured iteration renders the keyframes the
// scheduler (Sec. III-C-2) chose last without being captured again.
#include "gs_internal.h"

namespace gs {
namespace {

// blockIdx.y = batch slot; grid-stride over the slot's camera record, then
// its three colour planes, then its depth plane.
__global__ void __launch_bounds__(256) k_gather_views(
    const float* __restrict__ pool_cams, const float* __restrict__ pool_rgb,
    const float* __restrict__ pool_depth, const int32_t* __restrict__ sel, int32_t n_pool,
    int64_t pv, float* __restrict__ cams_out, float* __restrict__ rgb_out,
    float* __restrict__ depth_out) {
  const int b = blockIdx.y;
  const int32_t id = sel[b];
  if (id < 0 || id >= n_pool) return;  // slot left as it was
  constexpr int64_t C = GS_CAMERA_FLOATS;
  const int64_t per = C + 3 * pv + (pool_depth ? pv : 0);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per; e += stride) {
    if (e < C) {
      cams_out[b * C + e] = pool_cams[(int64_t)id * C + e];
    } else if (e < C + 3 * pv) {
      const int64_t k = e - C;
      rgb_out[b * 3 * pv + k] = pool_rgb[(int64_t)id * 3 * pv + k];
    } else {
      const int64_t k = e - C - 3 * pv;
      depth_out[b * pv + k] = pool_depth[(int64_t)id * pv + k];
    }
  }
}

}  // namespace

hipError_t launch_gather_views(const Plan& P, const gs_view_gather& g, float* cams_out,
                               float* rgb_out, float* depth_out, hipStream_t s) {
  const int64_t pv = (int64_t)P.vt.v[0].W * P.vt.v[0].H;
  const int64_t per = GS_CAMERA_FLOATS + 4 * pv;
  const unsigned gx = (unsigned)std::min<int64_t>((per + 255) / 256, 1024);
  hipLaunchKernelGGL(k_gather_views, dim3(gx, (unsigned)P.vt.n_views), dim3(256), 0, s,
                     g.pool_cams, g.pool_rgb, g.pool_depth, g.sel, g.n_pool, pv, cams_out,
                     rgb_out, depth_out);
  return hipGetLastError();
}

}  // namespace gs

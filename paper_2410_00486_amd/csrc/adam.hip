// a7: Adam over several parameter groups in one launch (the 3DGS optimiser,
// retained by the paper, Sec. IV-A), with the optional opacity regulariser
// of Eq. (10) folded into the gradient of the opacity-logit group.
// Bound by HBM: 28 bytes per parameter (p, g, m, v read; p, m, v written).
#include "gs_internal.h"

namespace gs {

constexpr int kAdamMaxGroups = 8;
constexpr int kAdamThreads = 256;
constexpr int kAdamVec = 4;  // float4 per thread

struct AdamGroupArg {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  int64_t block0;  // first block of this group
  float lr;
  int32_t reg;
  // optional: the gradient of element e is taken as zero unless
  // vis[e / per] != 0 (Gaussians without pairs, whose entries the one-view
  // projection backward leaves unwritten)
  const uint32_t* vis;
  int32_t per;
};

struct AdamArgs {
  AdamGroupArg grp[kAdamMaxGroups];
  int32_t n_groups;
  int32_t step;
  double beta1d, beta2d;  // for the bias corrections
  float beta1, beta2;     // multipliers of m and v
  float omb1, omb2;       // 1 - beta, formed in double
  float eps;
  float reg_scale;        // lambda_o / reg_count
  const int32_t* step_dev;
  // the iteration advanced *step_dev already and stored the factors of the
  // step; group k of this launch is group group0 + k there
  const AdamStepFactors* factors;
  int32_t group0;
  const int32_t* overflow;  // optional: a nonzero flag turns the launch into a no-op
  // optional: block 0 also reduces the forward's per-tile L1 partials of a
  // one-view iteration into *loss (the loss needs nothing after the forward)
  const float2* tile_loss;
  int32_t loss_tiles, loss_has_depth;
  double loss_pixels;
  float lambda_depth;
  float* loss;
};

namespace {

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, const AdamArgs& a,
                                         float step_size, float inv_bc2s, int reg) {
  if (reg) {
    const float o = 1.0f / (1.0f + expf(-p));
    g += a.reg_scale * o * (1.0f - o);
  }
  const float b1 = a.beta1, b2 = a.beta2, eps = a.eps;
  m = b1 * m + a.omb1 * g;
  v = b2 * v + a.omb2 * g * g;
  const float denom = sqrtf(v) * inv_bc2s + eps;
  p = p - step_size * (m / denom);
}

__global__ void __launch_bounds__(kAdamThreads) k_adam(AdamArgs a) {
  int gi = 0;
  while (gi + 1 < a.n_groups && (int64_t)blockIdx.x >= a.grp[gi + 1].block0) ++gi;
  const AdamGroupArg G = a.grp[gi];
  if (a.loss && blockIdx.x == 0)
    loss_reduce_view<kAdamThreads>(a.tile_loss, a.loss_tiles, a.loss_pixels, a.lambda_depth,
                                   a.loss_has_depth, a.loss);
  // the iteration's binning overflowed: its gradients are invalid, and the
  // parameters and moments are left as they are (the step counter was not
  // advanced either)
  if (a.overflow && *a.overflow != 0) return;
  float step_size, inv_bc2s;
  int step;
  if (a.factors) {
    step = a.factors->step;
    step_size = a.factors->step_size[a.group0 + gi];
    inv_bc2s = a.factors->inv_bc2s;
  } else {
    step = a.step_dev ? (*a.step_dev + 1) : a.step;
    const double bc1 = 1.0 - pow(a.beta1d, (double)step);
    const double bc2 = 1.0 - pow(a.beta2d, (double)step);
    step_size = (float)((double)G.lr / bc1);
    inv_bc2s = (float)(1.0 / sqrt(bc2));
  }
  // Odd steps walk the group's blocks backwards: the part of the state
  // touched last by the previous step is still in the last-level cache when
  // this one starts.  The order does not change any value.
  const int64_t gblocks = (G.n + kAdamThreads * kAdamVec - 1) / (kAdamThreads * kAdamVec);
  const int64_t lb = (int64_t)blockIdx.x - G.block0;
  const int64_t wb = (step & 1) ? gblocks - 1 - lb : lb;
  const int64_t e0 = wb * (kAdamThreads * kAdamVec) + (int64_t)threadIdx.x * kAdamVec;
  if (e0 + kAdamVec <= G.n) {
    // p, m, v first: they do not wait for the visibility lookup
    float4 p = *reinterpret_cast<float4*>(G.p + e0);
    float4 m = *reinterpret_cast<float4*>(G.m + e0);
    float4 v = *reinterpret_cast<float4*>(G.v + e0);
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (G.vis) {
      // visibility of the four elements' Gaussians (e0 is a multiple of 4)
      bool v0, v1, v2, v3;
      if (G.per == 1) {
        const uint4 t = *reinterpret_cast<const uint4*>(G.vis + e0);
        v0 = t.x != 0; v1 = t.y != 0; v2 = t.z != 0; v3 = t.w != 0;
      } else {
        // e0 = q0 per + r0; element e0 + i belongs to Gaussian q0 + (r0 + i) / per
        int64_t q0;
        if (G.n <= 0xFFFFFFFFll) {  // uniform: 32-bit division
          q0 = (int64_t)((uint32_t)e0 / (uint32_t)G.per);
        } else {
          q0 = e0 / G.per;
        }
        const int r0 = (int)(e0 - q0 * G.per);
        const int per = G.per;
        auto vis_at = [&](int i) {
          const int r = r0 + i;
          const int64_t q = q0 + (r >= per ? 1 : 0) + (r >= 2 * per ? 1 : 0) + (r >= 3 * per ? 1 : 0);
          return G.vis[q] != 0;
        };
        v0 = vis_at(0);
        v1 = vis_at(1);
        v2 = vis_at(2);
        v3 = vis_at(3);
      }
      if (v0 || v1 || v2 || v3) {
        const float4 gl = *reinterpret_cast<const float4*>(G.g + e0);
        g = make_float4(v0 ? gl.x : 0.f, v1 ? gl.y : 0.f, v2 ? gl.z : 0.f, v3 ? gl.w : 0.f);
      }
    } else {
      g = *reinterpret_cast<const float4*>(G.g + e0);
    }
    adam_one(p.x, g.x, m.x, v.x, a, step_size, inv_bc2s, G.reg);
    adam_one(p.y, g.y, m.y, v.y, a, step_size, inv_bc2s, G.reg);
    adam_one(p.z, g.z, m.z, v.z, a, step_size, inv_bc2s, G.reg);
    adam_one(p.w, g.w, m.w, v.w, a, step_size, inv_bc2s, G.reg);
    *reinterpret_cast<float4*>(G.p + e0) = p;
    *reinterpret_cast<float4*>(G.m + e0) = m;
    *reinterpret_cast<float4*>(G.v + e0) = v;
  } else {
    for (int64_t e = e0; e < G.n; ++e) {
      float p = G.p[e], m = G.m[e], v = G.v[e];
      const bool live = !G.vis || G.vis[e / G.per] != 0;
      adam_one(p, live ? G.g[e] : 0.0f, m, v, a, step_size, inv_bc2s, G.reg);
      G.p[e] = p;
      G.m[e] = m;
      G.v[e] = v;
    }
  }
}

__global__ void k_step_advance(int32_t* step_dev, const int32_t* overflow) {
  if (!overflow || *overflow == 0) *step_dev += 1;
}

}  // namespace

int64_t adam_blocks(int64_t n) {
  return (n + kAdamThreads * kAdamVec - 1) / (kAdamThreads * kAdamVec);
}

// vis / per: optional per-group gradient masks (see AdamGroupArg).
// overflow (optional): the pair-overflow flag of the iteration; when set on
// the device, the launch changes no parameter, moment or step counter.
// fold (optional): the iteration advanced step_dev already, and/or the
// forward's loss reduction rides on block 0.
hipError_t launch_adam(const gs_param_group* groups, int n_groups, int step, double beta1,
                       double beta2, double eps, double lambda_o, int64_t reg_count,
                       int32_t* step_dev, hipStream_t s, const uint32_t* const* vis,
                       const int32_t* per, const int32_t* overflow, const AdamFold* fold) {
  for (int base = 0; base < n_groups; base += kAdamMaxGroups) {
    AdamArgs a{};
    const int ng = n_groups - base < kAdamMaxGroups ? n_groups - base : kAdamMaxGroups;
    int64_t blocks = 0;
    for (int k = 0; k < ng; ++k) {
      const gs_param_group& G = groups[base + k];
      a.grp[k] = AdamGroupArg{G.p, G.g, G.m, G.v, G.n, blocks, G.lr, G.opacity_reg,
                              vis ? vis[base + k] : nullptr, per ? per[base + k] : 1};
      blocks += adam_blocks(G.n);
    }
    a.n_groups = ng;
    a.step = step;
    a.beta1d = beta1;
    a.beta2d = beta2;
    a.beta1 = (float)beta1;
    a.beta2 = (float)beta2;
    a.omb1 = (float)(1.0 - beta1);
    a.omb2 = (float)(1.0 - beta2);
    a.eps = (float)eps;
    a.reg_scale = (lambda_o != 0.0 && reg_count > 0) ? (float)(lambda_o / (double)reg_count) : 0.0f;
    if (a.reg_scale == 0.0f)
      for (int k = 0; k < ng; ++k) a.grp[k].reg = 0;
    a.step_dev = step_dev;
    a.factors = (fold && fold->step_taken) ? fold->factors : nullptr;
    a.group0 = base;
    a.overflow = overflow;
    if (fold && fold->loss && base == 0) {
      a.tile_loss = fold->tile_loss;
      a.loss_tiles = fold->loss_tiles;
      a.loss_has_depth = fold->loss_has_depth;
      a.loss_pixels = fold->loss_pixels;
      a.lambda_depth = fold->lambda_depth;
      a.loss = fold->loss;
    }
    if (blocks > 0) hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(kAdamThreads), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (step_dev && !(fold && fold->step_taken)) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, s, step_dev, overflow);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace gs

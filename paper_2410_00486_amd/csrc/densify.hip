// Adaptive densification and opacity pruning (CaRtGS Sec. IV-A: densify every
// 500 iterations with a positional-gradient threshold, remove Gaussians with
// opacity below a threshold; clone / split as in 3DGS).
//
// gs_grad_stats: per Gaussian and view, the 2D mean gradient is the fixed-
// order sum of its pair partials (the same slots the projection backward
// reads); its norm in normalised device coordinates is added to `accum` and
// the visibility to `denom`.
//
// gs_densify_prune: per Gaussian an output count (0 pruned, 1 kept, 2 cloned
// or split), an exclusive scan of the counts, and a scatter that writes the
// new parameters and Adam moments in input order.  Split children use the
// caller's standard normal draws.  The new count is written to the device;
// nothing is written past the output capacity.
#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kDThreads = 256;
constexpr int kDItems = 8;
constexpr int kDTile = kDThreads * kDItems;

__global__ void __launch_bounds__(256) k_grad_stats(
    const uint32_t* __restrict__ tt, const uint32_t* __restrict__ poff,
    const float* __restrict__ grad_pair, const int32_t* __restrict__ fl, int64_t n, ViewTable vt,
    float* __restrict__ accum, float* __restrict__ denom) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || fl[F_OVERFLOW]) return;
  float a = 0.0f, d = 0.0f;
  for (int v = 0; v < vt.n_views; ++v) {
    const int64_t ri = (int64_t)v * n + i;
    const uint32_t c = tt[ri];
    if (c == 0) continue;
    const float* gp = grad_pair + (int64_t)poff[ri] * kPairGrad;
    double gx = 0.0, gy = 0.0;
    uint32_t k = 0;
    for (; k + 8 <= c; k += 8) {  // eight loads in flight, additions in order
      float2 m[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        m[u] = *reinterpret_cast<const float2*>(gp + (int64_t)(k + u) * kPairGrad + 8);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        gx += m[u].x;
        gy += m[u].y;
      }
    }
    for (; k < c; ++k) {
      gx += gp[(int64_t)k * kPairGrad + 8];
      gy += gp[(int64_t)k * kPairGrad + 9];
    }
    const double nx = gx * 0.5 * vt.v[v].W, ny = gy * 0.5 * vt.v[v].H;
    a += (float)sqrt(nx * nx + ny * ny);
    d += 1.0f;
  }
  accum[i] += a;
  denom[i] += d;
}

struct DensifyCfg {
  float tau_p, eps_alpha, percent_dense, extent;
};

__device__ __forceinline__ int out_count(const float* logits, const float* log_scales,
                                         const float* accum, const float* denom, int64_t i,
                                         const DensifyCfg& c, bool* split) {
  const float o = 1.0f / (1.0f + expf(-logits[i]));
  *split = false;
  if (!(o >= c.eps_alpha)) return 0;
  const float dn = denom[i];
  const bool sel = dn > 0.0f && accum[i] / dn >= c.tau_p;
  if (!sel) return 1;
  const float smax = expf(fmaxf(log_scales[3 * i], fmaxf(log_scales[3 * i + 1], log_scales[3 * i + 2])));
  *split = smax > c.percent_dense * c.extent;
  return 2;
}

__global__ void __launch_bounds__(kDThreads) k_densify_count(
    const float* __restrict__ logits, const float* __restrict__ log_scales,
    const float* __restrict__ accum, const float* __restrict__ denom, int64_t n, DensifyCfg cfg,
    uint32_t* __restrict__ offs, uint64_t* __restrict__ btot) {
  __shared__ uint32_t wsum[kDThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kDTile + (int64_t)threadIdx.x * kDItems;
  uint32_t c[kDItems];
  uint32_t s = 0;
  for (int k = 0; k < kDItems; ++k) {
    const int64_t i = base + k;
    bool sp;
    c[k] = i < n ? (uint32_t)out_count(logits, log_scales, accum, denom, i, cfg, &sp) : 0u;
    s += c[k];
  }
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint32_t incl = s;
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (int k = 0; k < w; ++k) woff += wsum[k];
  uint32_t run = woff + incl - s;
  for (int k = 0; k < kDItems; ++k) {
    const int64_t i = base + k;
    if (i < n) offs[i] = run;
    run += c[k];
  }
  if (threadIdx.x == kDThreads - 1) btot[blockIdx.x] = run;
}

__global__ void __launch_bounds__(1024) k_densify_totals(uint64_t* __restrict__ btot,
                                                         int64_t nblocks,
                                                         int32_t* __restrict__ n_out) {
  __shared__ uint64_t wsum[1024 / kWave];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (int64_t base = 0; base < nblocks; base += 1024) {
    const int64_t idx = base + threadIdx.x;
    const uint64_t x = idx < nblocks ? btot[idx] : 0ull;
    uint64_t incl = x;
    for (int o = 1; o < kWave; o <<= 1) {
      const uint64_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t woff = carry;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    if (idx < nblocks) btot[idx] = woff + incl - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry = woff + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_out = (int32_t)carry;
}

struct DensifyIO {
  const float *p_mean, *p_ls, *p_q, *p_op, *p_sh;
  const float *m_mean, *m_ls, *m_q, *m_op, *m_sh;
  const float *v_mean, *v_ls, *v_q, *v_op, *v_sh;
  float *o_mean, *o_ls, *o_q, *o_op, *o_sh;
  float *om_mean, *om_ls, *om_q, *om_op, *om_sh;
  float *ov_mean, *ov_ls, *ov_q, *ov_op, *ov_sh;
};

// Copy Gaussian i (parameters and, when keep_state, moments) to slot o.
__device__ __forceinline__ void put(const DensifyIO& io, int K3, int64_t i, int64_t o,
                                    bool keep_state) {
  for (int k = 0; k < 3; ++k) {
    io.o_mean[3 * o + k] = io.p_mean[3 * i + k];
    io.o_ls[3 * o + k] = io.p_ls[3 * i + k];
    io.om_mean[3 * o + k] = keep_state ? io.m_mean[3 * i + k] : 0.0f;
    io.ov_mean[3 * o + k] = keep_state ? io.v_mean[3 * i + k] : 0.0f;
    io.om_ls[3 * o + k] = keep_state ? io.m_ls[3 * i + k] : 0.0f;
    io.ov_ls[3 * o + k] = keep_state ? io.v_ls[3 * i + k] : 0.0f;
  }
  for (int k = 0; k < 4; ++k) {
    io.o_q[4 * o + k] = io.p_q[4 * i + k];
    io.om_q[4 * o + k] = keep_state ? io.m_q[4 * i + k] : 0.0f;
    io.ov_q[4 * o + k] = keep_state ? io.v_q[4 * i + k] : 0.0f;
  }
  io.o_op[o] = io.p_op[i];
  io.om_op[o] = keep_state ? io.m_op[i] : 0.0f;
  io.ov_op[o] = keep_state ? io.v_op[i] : 0.0f;
  for (int k = 0; k < K3; ++k) {
    io.o_sh[(int64_t)K3 * o + k] = io.p_sh[(int64_t)K3 * i + k];
    io.om_sh[(int64_t)K3 * o + k] = keep_state ? io.m_sh[(int64_t)K3 * i + k] : 0.0f;
    io.ov_sh[(int64_t)K3 * o + k] = keep_state ? io.v_sh[(int64_t)K3 * i + k] : 0.0f;
  }
}

__global__ void __launch_bounds__(256) k_densify_write(
    DensifyIO io, int K3, const float* __restrict__ accum, const float* __restrict__ denom,
    const float* __restrict__ normals, int64_t n, DensifyCfg cfg,
    const uint32_t* __restrict__ offs, const uint64_t* __restrict__ bpre, int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool split;
  const int c = out_count(io.p_op, io.p_ls, accum, denom, i, cfg, &split);
  if (c == 0) return;
  const int64_t o = (int64_t)offs[i] + (int64_t)bpre[i / kDTile];
  if (o + c > cap) return;
  if (c == 1 || !split) {
    put(io, K3, i, o, true);
    if (c == 2) put(io, K3, i, o + 1, false);
    return;
  }
  // split: two children with means p + R (s * n_k) and scales s / 1.6
  double q[4] = {io.p_q[4 * i], io.p_q[4 * i + 1], io.p_q[4 * i + 2], io.p_q[4 * i + 3]};
  const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] /= qn;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                       2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                       2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  const double s[3] = {exp((double)io.p_ls[3 * i]), exp((double)io.p_ls[3 * i + 1]),
                       exp((double)io.p_ls[3 * i + 2])};
  for (int ch = 0; ch < 2; ++ch) {
    const int64_t oc = o + ch;
    put(io, K3, i, oc, false);
    const float* nk = normals + 6 * i + 3 * ch;
    const double d[3] = {s[0] * nk[0], s[1] * nk[1], s[2] * nk[2]};
    for (int r = 0; r < 3; ++r)
      io.o_mean[3 * oc + r] =
          (float)((double)io.p_mean[3 * i + r] + R[3 * r] * d[0] + R[3 * r + 1] * d[1] + R[3 * r + 2] * d[2]);
    for (int r = 0; r < 3; ++r) io.o_ls[3 * oc + r] = (float)((double)io.p_ls[3 * i + r] - log(1.6));
  }
}

}  // namespace

size_t densify_tmp_bytes(int64_t n) {
  const int64_t nb = (n + kDTile - 1) / kDTile;
  return (size_t)(n + 64) * 4 + (size_t)(nb + 8) * 8 + 256;
}

hipError_t launch_grad_stats(const Plan& P, void* ws, float* accum, float* denom, hipStream_t s) {
  if (P.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_stats, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, s,
                     ws_at<uint32_t>(ws, P.off_tt), ws_at<uint32_t>(ws, P.off_poff),
                     ws_at<float>(ws, P.off_grad_pair), ws_at<int32_t>(ws, P.off_flags), P.n,
                     P.vt, accum, denom);
  return hipGetLastError();
}

hipError_t launch_densify(const gs_gaussians& g, const gs_gaussian_grads& m,
                          const gs_gaussian_grads& v, const float* accum, const float* denom,
                          const float* normals, float tau_p, float eps_alpha, float percent_dense,
                          float extent, const gs_gaussian_grads& out, const gs_gaussian_grads& out_m,
                          const gs_gaussian_grads& out_v, int64_t cap, int32_t* n_out, void* tmp,
                          hipStream_t s) {
  const int64_t n = g.n;
  const int64_t nb = (n + kDTile - 1) / kDTile;
  uint32_t* offs = static_cast<uint32_t*>(tmp);
  uint64_t* btot = reinterpret_cast<uint64_t*>(static_cast<char*>(tmp) + (((size_t)(n + 64) * 4 + 255) / 256) * 256);
  const DensifyCfg cfg{tau_p, eps_alpha, percent_dense, extent};
  if (nb > 0)
    hipLaunchKernelGGL(k_densify_count, dim3((unsigned)nb), dim3(kDThreads), 0, s, g.opacity_logits,
                       g.log_scales, accum, denom, n, cfg, offs, btot);
  hipLaunchKernelGGL(k_densify_totals, dim3(1), dim3(1024), 0, s, btot, nb, n_out);
  if (n > 0) {
    DensifyIO io{g.means, g.log_scales, g.quats, g.opacity_logits, g.sh,
                 m.means, m.log_scales, m.quats, m.opacity_logits, m.sh,
                 v.means, v.log_scales, v.quats, v.opacity_logits, v.sh,
                 out.means, out.log_scales, out.quats, out.opacity_logits, out.sh,
                 out_m.means, out_m.log_scales, out_m.quats, out_m.opacity_logits, out_m.sh,
                 out_v.means, out_v.log_scales, out_v.quats, out_v.opacity_logits, out_v.sh};
    const int K3 = 3 * (g.sh_degree + 1) * (g.sh_degree + 1);
    hipLaunchKernelGGL(k_densify_write, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, io, K3,
                       accum, denom, normals, n, cfg, offs, btot, cap);
  }
  return hipGetLastError();
}

}  // namespace gs

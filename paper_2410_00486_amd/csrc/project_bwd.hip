// a6: from per-pair 2D gradients to parameter and camera gradients.  One
// thread per Gaussian loops over the views: it sums the partials of its own
// (view, tile) pairs -- contiguous in generation order -- in a fixed order,
// recomputes the view's projection in FP64 and applies the chain rule
// through conic -> EWA covariance -> Jacobian -> camera-space mean, the 3D
// covariance (scale, rotation), the SH colour and the view direction, and
// the opacity sigmoid.  Without a camera tangent two threads (in two
// wavefronts of one workgroup) share a Gaussian, one for the projection
// chain and one for the colour chain.  Camera tangents (rho, phi) for a left
// perturbation of each pose are reduced per workgroup (fixed order) and then
// per view.
#include <type_traits>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr double kSH0 = 0.28209479177387814;
constexpr double kSH1 = 0.4886025119029199;
constexpr double kSH2a = 1.0925484305920792;
constexpr double kSH2b = 0.31539156525252005;
constexpr double kSH2c = 0.5462742152960396;
constexpr double kSH3a = 0.5900435899266435;
constexpr double kSH3b = 2.890611442640554;
constexpr double kSH3c = 0.4570457994644658;
constexpr double kSH3d = 0.3731763325901154;
constexpr double kSH3e = 1.445305721320277;

// For each basis function k up to DEG: Y_k and its gradient as a polynomial
// in (x, y, z) are formed in place, the SH-coefficient gradient Y_k * gcr is
// added to gsh[], and w_k grad Y_k (w_k = sum_ch gcr_ch SH_k,ch) to gd.  The
// coefficients shv[] and gradients gsh[] are registers: the caller loads
// and stores them in batches, so no memory round trip sits in the chain.
template <int DEG>
__device__ __forceinline__ void sh_backward(double x, double y, double z, const double* gcr,
                                            const float* shv, float* gsh, double& gx,
                                            double& gy, double& gz) {
  const double xx = x * x, yy = y * y, zz = z * z;
  auto term = [&](int k, double Yk, double dx, double dy, double dz) {
    double w = 0.0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      w += gcr[ch] * (double)shv[3 * k + ch];
      gsh[3 * k + ch] += (float)(Yk * gcr[ch]);
    }
    gx += w * dx;
    gy += w * dy;
    gz += w * dz;
  };
  term(0, kSH0, 0.0, 0.0, 0.0);
  if (DEG >= 1) {
    term(1, -kSH1 * y, 0.0, -kSH1, 0.0);
    term(2, kSH1 * z, 0.0, 0.0, kSH1);
    term(3, -kSH1 * x, -kSH1, 0.0, 0.0);
  }
  if (DEG >= 2) {
    term(4, kSH2a * x * y, kSH2a * y, kSH2a * x, 0.0);
    term(5, -kSH2a * y * z, 0.0, -kSH2a * z, -kSH2a * y);
    term(6, kSH2b * (2 * zz - xx - yy), -2 * kSH2b * x, -2 * kSH2b * y, 4 * kSH2b * z);
    term(7, -kSH2a * x * z, -kSH2a * z, 0.0, -kSH2a * x);
    term(8, kSH2c * (xx - yy), 2 * kSH2c * x, -2 * kSH2c * y, 0.0);
  }
  if (DEG >= 3) {
    term(9, -kSH3a * y * (3 * xx - yy), -6 * kSH3a * x * y, -kSH3a * (3 * xx - 3 * yy), 0.0);
    term(10, kSH3b * x * y * z, kSH3b * y * z, kSH3b * x * z, kSH3b * x * y);
    term(11, -kSH3c * y * (4 * zz - xx - yy), 2 * kSH3c * x * y, -kSH3c * (4 * zz - xx - 3 * yy),
         -8 * kSH3c * y * z);
    term(12, kSH3d * z * (2 * zz - 3 * xx - 3 * yy), -6 * kSH3d * x * z, -6 * kSH3d * y * z,
         kSH3d * (6 * zz - 3 * xx - 3 * yy));
    term(13, -kSH3c * x * (4 * zz - xx - yy), -kSH3c * (4 * zz - 3 * xx - yy), 2 * kSH3c * x * y,
         -8 * kSH3c * x * z);
    term(14, kSH3e * z * (xx - yy), 2 * kSH3e * x * z, -2 * kSH3e * y * z, kSH3e * (xx - yy));
    term(15, -kSH3a * x * (xx - 3 * yy), -kSH3a * (3 * xx - 3 * yy), 6 * kSH3a * x * y, 0.0);
  }
}

// Projection chain of one (view, Gaussian) record: from the summed pair
// partials g2[3..9] (depth, opacity, conic a b c, mean x y) and the world
// covariance S to the camera-space mean gradient gt and this view's term of
// dL/dSigma (dS: 00 11 22 01 02 12).  Also returns what the camera tangent
// needs (X = dL/dSigma', J's entries).
struct ProjTerm {
  double gt0, gt1, gt2;
  double dS[6];
  double X00, X01, X11, j00, j02, j11, j12;
};
__device__ __forceinline__ void proj_term(const double* W, double fx, double fy, double limx,
                                          double limy, double tx, double ty, double tz,
                                          double S00, double S01, double S02, double S11,
                                          double S12, double S22, const double* g2, ProjTerm& o) {
  const double ux = tx / tz, vy = ty / tz;
  const bool cu = (ux < -limx) || (ux > limx), cv = (vy < -limy) || (vy > limy);
  const double u = fmin(limx, fmax(-limx, ux)), wv = fmin(limy, fmax(-limy, vy));
  const double j00 = fx / tz, j02 = -fx * u / tz, j11 = fy / tz, j12 = -fy * wv / tz;
  const double a0 = j00 * W[0] + j02 * W[6], a1 = j00 * W[1] + j02 * W[7], a2 = j00 * W[2] + j02 * W[8];
  const double b0 = j11 * W[3] + j12 * W[6], b1 = j11 * W[4] + j12 * W[7], b2 = j11 * W[5] + j12 * W[8];
  const double Sa0 = S00 * a0 + S01 * a1 + S02 * a2, Sa1 = S01 * a0 + S11 * a1 + S12 * a2,
               Sa2 = S02 * a0 + S12 * a1 + S22 * a2;
  const double Sb0 = S00 * b0 + S01 * b1 + S02 * b2, Sb1 = S01 * b0 + S11 * b1 + S12 * b2,
               Sb2 = S02 * b0 + S12 * b1 + S22 * b2;
  const double A = a0 * Sa0 + a1 * Sa1 + a2 * Sa2 + 0.3;
  const double B = 0.5 * ((a0 * Sb0 + a1 * Sb1 + a2 * Sb2) + (b0 * Sa0 + b1 * Sa1 + b2 * Sa2));
  const double C = b0 * Sb0 + b1 * Sb1 + b2 * Sb2 + 0.3;
  const double det = A * C - B * B;
  const double ya = C / det, yb = -B / det, yc = A / det;  // conic
  // dL/dX = -Y G_Y Y with G_Y = [[ga, gb/2], [gb/2, gc]]
  const double ga = g2[5], gbh = 0.5 * g2[6], gc = g2[7];
  const double M00 = ya * ga + yb * gbh, M01 = ya * gbh + yb * gc;
  const double M10 = yb * ga + yc * gbh, M11 = yb * gbh + yc * gc;
  const double X00 = -(M00 * ya + M01 * yb);
  const double X01 = -(M00 * yb + M01 * yc);
  const double X11 = -(M10 * yb + M11 * yc);
  // G_Sigma += X00 a a^T + X01 (a b^T + b a^T) + X11 b b^T
  o.dS[0] = X00 * a0 * a0 + 2.0 * X01 * a0 * b0 + X11 * b0 * b0;
  o.dS[1] = X00 * a1 * a1 + 2.0 * X01 * a1 * b1 + X11 * b1 * b1;
  o.dS[2] = X00 * a2 * a2 + 2.0 * X01 * a2 * b2 + X11 * b2 * b2;
  o.dS[3] = X00 * a0 * a1 + X01 * (a0 * b1 + b0 * a1) + X11 * b0 * b1;
  o.dS[4] = X00 * a0 * a2 + X01 * (a0 * b2 + b0 * a2) + X11 * b0 * b2;
  o.dS[5] = X00 * a1 * a2 + X01 * (a1 * b2 + b1 * a2) + X11 * b1 * b2;
  // G_T2 rows: 2 (X00 Sa + X01 Sb), 2 (X01 Sa + X11 Sb);  G_J = G_T2 W^T
  const double r00 = 2 * (X00 * Sa0 + X01 * Sb0), r01 = 2 * (X00 * Sa1 + X01 * Sb1),
               r02 = 2 * (X00 * Sa2 + X01 * Sb2);
  const double r10 = 2 * (X01 * Sa0 + X11 * Sb0), r11 = 2 * (X01 * Sa1 + X11 * Sb1),
               r12 = 2 * (X01 * Sa2 + X11 * Sb2);
  const double GJ00 = r00 * W[0] + r01 * W[1] + r02 * W[2];
  const double GJ02 = r00 * W[6] + r01 * W[7] + r02 * W[8];
  const double GJ11 = r10 * W[3] + r11 * W[4] + r12 * W[5];
  const double GJ12 = r10 * W[6] + r11 * W[7] + r12 * W[8];
  const double tz2 = tz * tz, tz3 = tz2 * tz;
  double gt0 = 0, gt1 = 0, gt2;
  gt2 = -GJ00 * fx / tz2 - GJ11 * fy / tz2;
  if (!cu) { gt0 += -GJ02 * fx / tz2; gt2 += GJ02 * 2.0 * fx * tx / tz3; }
  else { gt2 += GJ02 * fx * u / tz2; }
  if (!cv) { gt1 += -GJ12 * fy / tz2; gt2 += GJ12 * 2.0 * fy * ty / tz3; }
  else { gt2 += GJ12 * fy * wv / tz2; }
  const double gmx = g2[8], gmy = g2[9];
  gt0 += gmx * fx / tz;
  gt1 += gmy * fy / tz;
  gt2 += -(gmx * fx * tx + gmy * fy * ty) / tz2 + g2[3];
  o.gt0 = gt0; o.gt1 = gt1; o.gt2 = gt2;
  o.X00 = X00; o.X01 = X01; o.X11 = X11;
  o.j00 = j00; o.j02 = j02; o.j11 = j11; o.j12 = j12;
}

// Colour chain of one record: SH-coefficient gradients added into gsh[] and
// the view-direction part gv of the mean gradient, from the colour partials
// g2[0..2] (channels clamped at 0 by the forward projection carry none).
template <int DEG>
__device__ __forceinline__ void colour_term(const double* W, double t0, double t1, double t2,
                                            const double* p, uint32_t cmask, const double* g2,
                                            const float* shv, float* gsh, double& gv0,
                                            double& gv1, double& gv2) {
  const double cxw = -(W[0] * t0 + W[3] * t1 + W[6] * t2);
  const double cyw = -(W[1] * t0 + W[4] * t1 + W[7] * t2);
  const double czw = -(W[2] * t0 + W[5] * t1 + W[8] * t2);
  const double dv0 = p[0] - cxw, dv1 = p[1] - cyw, dv2 = p[2] - czw;
  const double dist = sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
  const double d0 = dv0 / dist, d1 = dv1 / dist, d2 = dv2 / dist;
  double gcr[3];
  for (int ch = 0; ch < 3; ++ch) gcr[ch] = ((cmask >> ch) & 1u) ? 0.0 : g2[ch];
  double gd0 = 0, gd1 = 0, gd2 = 0;
  sh_backward<DEG>(d0, d1, d2, gcr, shv, gsh, gd0, gd1, gd2);
  const double dd = gd0 * d0 + gd1 * d1 + gd2 * d2;
  gv0 = (gd0 - dd * d0) / dist;
  gv1 = (gd1 - dd * d1) / dist;
  gv2 = (gd2 - dd * d2) / dist;
}

// COMPACT (one view): threads take the visible Gaussians from the list the
// binning wrote, in index order, so that the long chain runs on full
// wavefronts; the other Gaussians' gradients are zeroed beforehand.
// SPLIT (no pose gradient): the two wavefronts of a workgroup take the same
// 64 Gaussians, one the projection chain (mean, scale, rotation, opacity),
// the other the colour chain (SH coefficients and the view-direction part of
// the mean gradient, handed over in LDS after the views), so the two halves
// of each Gaussian's chain run side by side, each with its own registers.
// With one view (COMPACT) two more wavefronts join them for the sums of the
// pair partials: wavefront w sums the w-th quarter of each Gaussian's pairs
// (in pair order) into LDS and the chains add the four quarters in order, so
// a Gaussian with many pairs waits for a quarter of the memory round trips.
constexpr int kSumWaves = 4;
template <int DEG, bool POSE, bool COMPACT, bool SPLIT>
__global__ void __launch_bounds__((SPLIT && COMPACT) ? kSumWaves * kWave : kProjThreads) k_project_bwd(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, const float* __restrict__ cams, ViewTable vt,
    const Rec* __restrict__ recs, const uint32_t* __restrict__ tt, const uint32_t* __restrict__ poff,
    const float* __restrict__ grad_pair, const int32_t* __restrict__ fl,
    const uint32_t* __restrict__ vis_list, int accumulate,
    float* __restrict__ g_means, float* __restrict__ g_ls, float* __restrict__ g_q,
    float* __restrict__ g_logit, float* __restrict__ g_sh, double* __restrict__ pose_part,
    int64_t pose_stride) {
  static_assert(!(SPLIT && POSE), "the camera tangent needs both halves in one thread");
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int NW = kProjThreads / kWave;
  const bool overflow = fl[F_OVERFLOW] != 0;
  const int lane = lane_id();
  // wavefront role (SPLIT): 0 projection chain, 1 colour chain
  const int role = SPLIT ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)) : 0;
  const int64_t t0 = SPLIT ? (int64_t)blockIdx.x * kWave + lane
                           : (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
  bool valid;
  int64_t i;
  if (COMPACT) {
    const int64_t nv = overflow ? 0 : (int64_t)fl[F_VISIBLE];
    valid = t0 < nv;
    i = valid ? (int64_t)vis_list[t0] : 0;
  } else {
    valid = t0 < n;
    i = t0;
  }
  __shared__ double spose[NW][6];
  __shared__ double sgv[3][kWave];
  constexpr bool COOP = SPLIT && COMPACT;
  // COOP: the pair sums of the four quarters (ten partials each)
  __shared__ double ssum[COOP ? kSumWaves : 1][COOP ? 10 : 1][kWave];
  if constexpr (COOP) {
    const int w = role;  // every wavefront sums a quarter first
    const int64_t ig = valid ? i : 0;
    const uint32_t cnt = (valid && !overflow) ? tt[ig] : 0u;  // one view: record = Gaussian
    const uint32_t lo = (uint32_t)(((uint64_t)cnt * (uint32_t)w) / kSumWaves);
    const uint32_t hi = (uint32_t)(((uint64_t)cnt * (uint32_t)(w + 1)) / kSumWaves);
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (hi > lo) {
      const float* gpp = grad_pair + (int64_t)poff[ig] * kPairGrad;
      auto add = [&](const PairSlot& p) {
        s[0] += p.a.x; s[1] += p.a.y; s[2] += p.a.z; s[3] += p.a.w;
        s[4] += p.b.x; s[5] += p.b.y; s[6] += p.b.z; s[7] += p.b.w;
        s[8] += p.c.x; s[9] += p.c.y;
      };
      uint32_t k = lo;
      for (; k + 8 <= hi; k += 8) {
        PairSlot a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = load_pair(gpp, k + u);
#pragma unroll
        for (int u = 0; u < 8; ++u) add(a[u]);
      }
      for (; k < hi; ++k) add(load_pair(gpp, k));
    }
#pragma unroll
    for (int c = 0; c < 10; ++c) ssum[w][c][lane] = s[c];
    __syncthreads();
    if (w >= 2) {  // helpers: only the hand-over barrier of the chains is left
      __syncthreads();
      return;
    }
  }

  // Every per-Gaussian input is loaded at once, unconditionally (row 0 for
  // an idle thread; n > 0 whenever the kernel runs), so that the loads issue
  // together instead of one round trip each along the chain.
  const int64_t ic = valid ? i : 0;

  // DP: projection chain, DS: colour chain (both without SPLIT)
  auto run = [&](auto dp_tag, auto ds_tag) {
    constexpr bool DP = decltype(dp_tag)::value, DS = decltype(ds_tag)::value;
    const float mf0 = means[3 * ic], mf1 = means[3 * ic + 1], mf2 = means[3 * ic + 2];
    float qf0 = 0, qf1 = 0, qf2 = 0, qf3 = 0, lf0 = 0, lf1 = 0, lf2 = 0, logit = 0;
    if (DP) {
      qf0 = quats[4 * ic]; qf1 = quats[4 * ic + 1]; qf2 = quats[4 * ic + 2]; qf3 = quats[4 * ic + 3];
      lf0 = log_scales[3 * ic]; lf1 = log_scales[3 * ic + 1]; lf2 = log_scales[3 * ic + 2];
      logit = logits[ic];
    }
    // SH coefficients and their gradient in registers for the whole view
    // loop, loaded the same way
    constexpr int KS = DS ? K * 3 : 1;
    float shv[KS], gsh[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      shv[k] = DS ? sh[ic * (K * 3) + k] : 0.0f;
      gsh[k] = 0.0f;
    }

    // world covariance Sigma (view independent); its gradient is summed over
    // views and pushed through scale and rotation once, after the view loop
    double p[3] = {0, 0, 0};
    double S00 = 0, S01 = 0, S02 = 0, S11 = 0, S12 = 0, S22 = 0;
    if (valid) {
      p[0] = mf0; p[1] = mf1; p[2] = mf2;
    }
    if (DP && valid) {
      double q[4] = {qf0, qf1, qf2, qf3};
      const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      if (qn > 0.0)
        for (int k = 0; k < 4; ++k) q[k] /= qn;
      const double w = q[0], x = q[1], y = q[2], z = q[3];
      const double R00 = 1 - 2 * (y * y + z * z), R01 = 2 * (x * y - w * z), R02 = 2 * (x * z + w * y);
      const double R10 = 2 * (x * y + w * z), R11 = 1 - 2 * (x * x + z * z), R12 = 2 * (y * z - w * x);
      const double R20 = 2 * (x * z - w * y), R21 = 2 * (y * z + w * x), R22 = 1 - 2 * (x * x + y * y);
      const double s0 = exp(2.0 * (double)lf0), s1 = exp(2.0 * (double)lf1), s2 = exp(2.0 * (double)lf2);
      S00 = R00 * R00 * s0 + R01 * R01 * s1 + R02 * R02 * s2;
      S01 = R00 * R10 * s0 + R01 * R11 * s1 + R02 * R12 * s2;
      S02 = R00 * R20 * s0 + R01 * R21 * s1 + R02 * R22 * s2;
      S11 = R10 * R10 * s0 + R11 * R11 * s1 + R12 * R12 * s2;
      S12 = R10 * R20 * s0 + R11 * R21 * s1 + R12 * R22 * s2;
      S22 = R20 * R20 * s0 + R21 * R21 * s1 + R22 * R22 * s2;
    }
    double gp0 = 0, gp1 = 0, gp2 = 0, gop = 0;
    double GS00 = 0, GS01 = 0, GS02 = 0, GS11 = 0, GS12 = 0, GS22 = 0;

    for (int v = 0; v < vt.n_views; ++v) {
      const int64_t ri = (int64_t)v * n + ic;
      const uint32_t tt_v = tt[ri], poff_v = poff[ri];
      const uint32_t cmask = DS ? recs[ri].clamp : 0u;
      const uint32_t cnt = (valid && !overflow) ? tt_v : 0u;
      double pose[6] = {0, 0, 0, 0, 0, 0};
      if (cnt > 0) {
        // fixed-order sum of this (view, Gaussian)'s pair partials (the
        // colour chain needs the first three, the projection chain the rest)
        double g2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (COOP) {
#pragma unroll
          for (int c = 0; c < 10; ++c)
            if ((DS && c < 3) || (DP && c >= 3))
              g2[c] = ((ssum[0][c][lane] + ssum[1][c][lane]) + ssum[2][c][lane]) + ssum[3][c][lane];
        } else {
          const float* gpp = grad_pair + (int64_t)poff_v * kPairGrad;
          auto add = [&](const PairSlot& p) {
            if (DS) { g2[0] += p.a.x; g2[1] += p.a.y; g2[2] += p.a.z; }
            if (DP) {
              g2[3] += p.a.w;
              g2[4] += p.b.x; g2[5] += p.b.y; g2[6] += p.b.z; g2[7] += p.b.w;
              g2[8] += p.c.x; g2[9] += p.c.y;
            }
          };
          // (the colour chain alone reads the colour partials only)
          auto load = [&](uint32_t kk) {
            if (DP) return load_pair(gpp, kk);
            return PairSlot{load_pair_colour(gpp, kk), make_float4(0.f, 0.f, 0.f, 0.f),
                            make_float2(0.f, 0.f)};
          };
          // loads of eight pairs are issued before their (in-order) additions,
          // so a large Gaussian does not pay one memory round trip per tile
          uint32_t k = 0;
          for (; k + 8 <= cnt; k += 8) {
            PairSlot a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = load(k + u);
#pragma unroll
            for (int u = 0; u < 8; ++u) add(a[u]);
          }
          for (; k < cnt; ++k) add(load(k));
        }
        gop += g2[4];
        const float* c = cams + (int64_t)v * GS_CAMERA_FLOATS;
        const double fx = c[0], fy = c[1];
        double W[9];
        for (int k = 0; k < 9; ++k) W[k] = c[4 + k];
        const double t0 = c[13], t1 = c[14], t2 = c[15];
        const double tx = W[0] * p[0] + W[1] * p[1] + W[2] * p[2] + t0;
        const double ty = W[3] * p[0] + W[4] * p[1] + W[5] * p[2] + t1;
        const double tz = W[6] * p[0] + W[7] * p[1] + W[8] * p[2] + t2;
        double gt0 = 0, gt1 = 0, gt2 = 0;
        double j00 = 0, j02 = 0, j11 = 0, j12 = 0, X00 = 0, X01 = 0, X11 = 0;
        if (DP) {
          const double limx = 1.3 * (double)vt.v[v].W / (2.0 * fx);
          const double limy = 1.3 * (double)vt.v[v].H / (2.0 * fy);
          ProjTerm pt;
          proj_term(W, fx, fy, limx, limy, tx, ty, tz, S00, S01, S02, S11, S12, S22, g2, pt);
          GS00 += pt.dS[0];
          GS11 += pt.dS[1];
          GS22 += pt.dS[2];
          GS01 += pt.dS[3];
          GS02 += pt.dS[4];
          GS12 += pt.dS[5];
          gt0 = pt.gt0; gt1 = pt.gt1; gt2 = pt.gt2;
          X00 = pt.X00; X01 = pt.X01; X11 = pt.X11;
          j00 = pt.j00; j02 = pt.j02; j11 = pt.j11; j12 = pt.j12;
        }

        double gv0 = 0, gv1 = 0, gv2 = 0;
        if (DS) colour_term<DEG>(W, t0, t1, t2, p, cmask, g2, shv, gsh, gv0, gv1, gv2);
        // mean: W^T g_t + g_v (the colour wavefront of SPLIT sums g_v alone)
        gp0 += W[0] * gt0 + W[3] * gt1 + W[6] * gt2 + gv0;
        gp1 += W[1] * gt0 + W[4] * gt1 + W[7] * gt2 + gv1;
        gp2 += W[2] * gt0 + W[5] * gt1 + W[8] * gt2 + gv2;
        if (POSE) {
          // camera tangent: rho = g_t + W g_v;  phi = t x g_t - 2 axial(Sc Gc - Gc Sc)
          pose[0] = gt0 + W[0] * gv0 + W[1] * gv1 + W[2] * gv2;
          pose[1] = gt1 + W[3] * gv0 + W[4] * gv1 + W[5] * gv2;
          pose[2] = gt2 + W[6] * gv0 + W[7] * gv1 + W[8] * gv2;
          pose[3] = ty * gt2 - tz * gt1;
          pose[4] = tz * gt0 - tx * gt2;
          pose[5] = tx * gt1 - ty * gt0;
          const double Sw[3][3] = {{S00, S01, S02}, {S01, S11, S12}, {S02, S12, S22}};
          double WS[3][3], Sc[3][3];
          for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc)
              WS[r][cc] = W[3 * r] * Sw[0][cc] + W[3 * r + 1] * Sw[1][cc] + W[3 * r + 2] * Sw[2][cc];
          for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc)
              Sc[r][cc] = WS[r][0] * W[3 * cc] + WS[r][1] * W[3 * cc + 1] + WS[r][2] * W[3 * cc + 2];
          const double jr0[3] = {j00, 0.0, j02}, jr1[3] = {0.0, j11, j12};
          double Gc[3][3];
          for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc)
              Gc[r][cc] = X00 * jr0[r] * jr0[cc] + X01 * (jr0[r] * jr1[cc] + jr1[r] * jr0[cc]) + X11 * jr1[r] * jr1[cc];
          double A21 = 0, A02 = 0, A10 = 0;
          for (int k = 0; k < 3; ++k) {
            A21 += Sc[2][k] * Gc[k][1] - Gc[2][k] * Sc[k][1];
            A02 += Sc[0][k] * Gc[k][2] - Gc[0][k] * Sc[k][2];
            A10 += Sc[1][k] * Gc[k][0] - Gc[1][k] * Sc[k][0];
          }
          pose[3] -= 2.0 * A21;
          pose[4] -= 2.0 * A02;
          pose[5] -= 2.0 * A10;
        }
      }
      if (POSE) {
        // workgroup sum of the camera tangent for this view, fixed order
        const int w = threadIdx.x / kWave;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const double sum = wave_sum(pose[k]);
          if (lane == 0) spose[w][k] = sum;
        }
        __syncthreads();
        if (threadIdx.x < 6) {
          double acc = 0.0;
          for (int ww = 0; ww < NW; ++ww) acc += spose[ww][threadIdx.x];
          pose_part[((int64_t)v * pose_stride + blockIdx.x) * 6 + threadIdx.x] = acc;
        }
        __syncthreads();
      }
    }

    if (DS && valid) {
      // SH gradients: sums over the views in registers, one batch of stores
      // (zeros for a Gaussian without pairs)
      float* gdst = g_sh + i * (K * 3);
      if (accumulate) {
        float old[KS];
#pragma unroll
        for (int k = 0; k < KS; ++k) old[k] = gdst[k];
#pragma unroll
        for (int k = 0; k < KS; ++k) gdst[k] = old[k] + gsh[k];
      } else {
#pragma unroll
        for (int k = 0; k < KS; ++k) gdst[k] = gsh[k];
      }
    }
    if (SPLIT) {
      // hand-over of the view-direction part of the mean gradient: one
      // barrier in each wavefront's path
      if (!DP) {
        sgv[0][lane] = gp0;
        sgv[1][lane] = gp1;
        sgv[2][lane] = gp2;
        __syncthreads();
        return;
      }
      __syncthreads();
      gp0 += sgv[0][lane];
      gp1 += sgv[1][lane];
      gp2 += sgv[2][lane];
    }
    if (!DP || !valid) return;
    // Sigma = M M^T, M = R diag(s):  g_l_j = 2 s_j^2 R_j^T G R_j,
    // G_R[:, j] = 2 s_j^2 G R_j, then through the normalised quaternion
    double q[4] = {qf0, qf1, qf2, qf3};
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (qn > 0.0)
      for (int k = 0; k < 4; ++k) q[k] /= qn;
    const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
    const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                         2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                         2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    double GR[9], gl[3];
    for (int j = 0; j < 3; ++j) {
      const double Rj0 = R[j], Rj1 = R[3 + j], Rj2 = R[6 + j];
      const double G0 = GS00 * Rj0 + GS01 * Rj1 + GS02 * Rj2;
      const double G1 = GS01 * Rj0 + GS11 * Rj1 + GS12 * Rj2;
      const double G2 = GS02 * Rj0 + GS12 * Rj1 + GS22 * Rj2;
      const double s2 = exp(2.0 * (double)(j == 0 ? lf0 : (j == 1 ? lf1 : lf2)));
      gl[j] = 2.0 * s2 * (Rj0 * G0 + Rj1 * G1 + Rj2 * G2);
      GR[j] = 2.0 * s2 * G0;
      GR[3 + j] = 2.0 * s2 * G1;
      GR[6 + j] = 2.0 * s2 * G2;
    }
    const double dw = GR[1] * (-2 * qz) + GR[2] * (2 * qy) + GR[3] * (2 * qz) + GR[5] * (-2 * qx) +
                      GR[6] * (-2 * qy) + GR[7] * (2 * qx);
    const double dx = GR[1] * (2 * qy) + GR[2] * (2 * qz) + GR[3] * (2 * qy) + GR[4] * (-4 * qx) +
                      GR[5] * (-2 * qw) + GR[6] * (2 * qz) + GR[7] * (2 * qw) + GR[8] * (-4 * qx);
    const double dy = GR[0] * (-4 * qy) + GR[1] * (2 * qx) + GR[2] * (2 * qw) + GR[3] * (2 * qx) +
                      GR[5] * (2 * qz) + GR[6] * (-2 * qw) + GR[7] * (2 * qz) + GR[8] * (-4 * qy);
    const double dz = GR[0] * (-4 * qz) + GR[1] * (-2 * qw) + GR[2] * (2 * qx) + GR[3] * (2 * qw) +
                      GR[4] * (-4 * qz) + GR[5] * (2 * qy) + GR[6] * (2 * qx) + GR[7] * (2 * qy);
    const double dot = dw * qw + dx * qx + dy * qy + dz * qz;
    const double o = 1.0 / (1.0 + exp(-(double)logit));
    auto put = [&](float* dst, double val) { *dst = accumulate ? *dst + (float)val : (float)val; };
    put(&g_means[3 * i], gp0);
    put(&g_means[3 * i + 1], gp1);
    put(&g_means[3 * i + 2], gp2);
    for (int r = 0; r < 3; ++r) put(&g_ls[3 * i + r], gl[r]);
    const double qnn = qn > 0.0 ? qn : 1.0;
    put(&g_q[4 * i], (dw - dot * qw) / qnn);
    put(&g_q[4 * i + 1], (dx - dot * qx) / qnn);
    put(&g_q[4 * i + 2], (dy - dot * qy) / qnn);
    put(&g_q[4 * i + 3], (dz - dot * qz) / qnn);
    put(&g_logit[i], gop * o * (1.0 - o));
  };
  using T = std::true_type;
  using F = std::false_type;
  if (!SPLIT) run(T{}, T{});
  else if (role == 0) run(T{}, F{});
  else run(F{}, T{});
}

// Several views, no camera tangent: two launches, each on full wavefronts
// whatever the visibility pattern.
//   k_project_rec: one thread per visible (view, Gaussian) record (the
//     visible list): the record's pair partials summed in pair order, then
//     that view's projection chain; the record's terms (mean and covariance
//     parts, opacity), its summed colour partials and clamp bits go to the
//     record's slot.
//   k_project_gauss: one thread per Gaussian: its records' terms added in
//     view order, the colour chain of each view (SH coefficients held in
//     registers), then the covariance -> scale / rotation chain.
// The operations and their order are those of one thread looping over the
// views (projection sums, colour sums, then their total), so the gradients
// do not depend on how the records are spread over threads.
constexpr int kTermWords = 14;  // doubles per record slot (112 bytes)
constexpr int kRecThreads = 256;
constexpr int kGaussThreads = 128;

template <int DEG>
__global__ void __launch_bounds__(kRecThreads) k_project_rec(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, int64_t n, const float* __restrict__ cams, ViewTable vt,
    const uint32_t* __restrict__ tt, const uint32_t* __restrict__ poff,
    const float* __restrict__ grad_pair, const int32_t* __restrict__ fl,
    const uint32_t* __restrict__ vis_list, const uint32_t* __restrict__ vis_clamp,
    double* __restrict__ terms) {
  const int64_t j = (int64_t)blockIdx.x * kRecThreads + threadIdx.x;
  const int64_t nv = fl[F_OVERFLOW] ? 0 : (int64_t)fl[F_VISIBLE];
  if (j >= nv) return;
  const uint32_t ri = vis_list[j];
  const int v = (int)(ri / (uint64_t)n);
  const int64_t i = (int64_t)ri - (int64_t)v * n;
  const uint32_t np = tt[ri];
  const float* gp = grad_pair + (int64_t)poff[ri] * kPairGrad;
  // fixed-order sums of the pair partials: colour 0..2, projection 3..9
  double g2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  auto add = [&](const PairSlot& p) {
    g2[0] += p.a.x; g2[1] += p.a.y; g2[2] += p.a.z; g2[3] += p.a.w;
    g2[4] += p.b.x; g2[5] += p.b.y; g2[6] += p.b.z; g2[7] += p.b.w;
    g2[8] += p.c.x; g2[9] += p.c.y;
  };
  uint32_t q = 0;
  for (; q + 4 <= np; q += 4) {
    PairSlot a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = load_pair(gp, q + u);
#pragma unroll
    for (int u = 0; u < 4; ++u) add(a[u]);
  }
  for (; q < np; ++q) add(load_pair(gp, q));
  // world covariance of the Gaussian
  double qv[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
  const double qn = sqrt(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]);
  if (qn > 0.0)
    for (int k = 0; k < 4; ++k) qv[k] /= qn;
  const double w = qv[0], x = qv[1], y = qv[2], z = qv[3];
  const double R00 = 1 - 2 * (y * y + z * z), R01 = 2 * (x * y - w * z), R02 = 2 * (x * z + w * y);
  const double R10 = 2 * (x * y + w * z), R11 = 1 - 2 * (x * x + z * z), R12 = 2 * (y * z - w * x);
  const double R20 = 2 * (x * z - w * y), R21 = 2 * (y * z + w * x), R22 = 1 - 2 * (x * x + y * y);
  const double s0 = exp(2.0 * (double)log_scales[3 * i]);
  const double s1 = exp(2.0 * (double)log_scales[3 * i + 1]);
  const double s2 = exp(2.0 * (double)log_scales[3 * i + 2]);
  const double S00 = R00 * R00 * s0 + R01 * R01 * s1 + R02 * R02 * s2;
  const double S01 = R00 * R10 * s0 + R01 * R11 * s1 + R02 * R12 * s2;
  const double S02 = R00 * R20 * s0 + R01 * R21 * s1 + R02 * R22 * s2;
  const double S11 = R10 * R10 * s0 + R11 * R11 * s1 + R12 * R12 * s2;
  const double S12 = R10 * R20 * s0 + R11 * R21 * s1 + R12 * R22 * s2;
  const double S22 = R20 * R20 * s0 + R21 * R21 * s1 + R22 * R22 * s2;
  const float* c = cams + (int64_t)v * GS_CAMERA_FLOATS;
  const double fx = c[0], fy = c[1];
  double W[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) W[e] = c[4 + e];
  const double limx = 1.3 * (double)vt.v[v].W / (2.0 * (double)c[0]);
  const double limy = 1.3 * (double)vt.v[v].H / (2.0 * (double)c[1]);
  const double p0 = means[3 * i], p1 = means[3 * i + 1], p2 = means[3 * i + 2];
  const double tx = W[0] * p0 + W[1] * p1 + W[2] * p2 + c[13];
  const double ty = W[3] * p0 + W[4] * p1 + W[5] * p2 + c[14];
  const double tz = W[6] * p0 + W[7] * p1 + W[8] * p2 + c[15];
  ProjTerm pt;
  proj_term(W, fx, fy, limx, limy, tx, ty, tz, S00, S01, S02, S11, S12, S22, g2, pt);
  double o[kTermWords];
  o[0] = W[0] * pt.gt0 + W[3] * pt.gt1 + W[6] * pt.gt2 + 0.0;
  o[1] = W[1] * pt.gt0 + W[4] * pt.gt1 + W[7] * pt.gt2 + 0.0;
  o[2] = W[2] * pt.gt0 + W[5] * pt.gt1 + W[8] * pt.gt2 + 0.0;
#pragma unroll
  for (int e = 0; e < 6; ++e) o[3 + e] = pt.dS[e];
  o[9] = g2[4];
  o[10] = g2[0];
  o[11] = g2[1];
  o[12] = g2[2];
  o[13] = (double)vis_clamp[j];
  double2* dst = reinterpret_cast<double2*>(terms + (int64_t)ri * kTermWords);
#pragma unroll
  for (int e = 0; e < kTermWords / 2; ++e) dst[e] = make_double2(o[2 * e], o[2 * e + 1]);
}

// Projection half per Gaussian: the records' mean, covariance and opacity
// terms added in view order, then the covariance -> scale / rotation chain;
// the mean sum and the mask of views that see the Gaussian wait in gp_tmp
// (four words per Gaussian) for the colour half.
__global__ void __launch_bounds__(kGaussThreads) k_project_gauss(
    const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ logits, int64_t n, int n_views, const uint32_t* __restrict__ tt,
    const double* __restrict__ terms, const int32_t* __restrict__ fl, int accumulate,
    double* __restrict__ gp_tmp, float* __restrict__ g_ls, float* __restrict__ g_q,
    float* __restrict__ g_logit) {
  const int64_t i = (int64_t)blockIdx.x * kGaussThreads + threadIdx.x;
  if (i >= n) return;
  const bool overflow = fl[F_OVERFLOW] != 0;
  uint64_t mask = 0;
  if (!overflow)
    for (int v = 0; v < n_views; ++v)
      if (tt[(int64_t)v * n + i] > 0u) mask |= 1ull << v;
  double gp0 = 0, gp1 = 0, gp2 = 0, gop = 0;
  double GS00 = 0, GS01 = 0, GS02 = 0, GS11 = 0, GS12 = 0, GS22 = 0;
  for (uint64_t m = mask; m; m &= m - 1) {
    const int v = __builtin_ctzll(m);
    const double2* src = reinterpret_cast<const double2*>(terms + ((int64_t)v * n + i) * kTermWords);
    const double2 a = src[0], b = src[1], c = src[2], d = src[3], e = src[4];
    gp0 += a.x;
    gp1 += a.y;
    gp2 += b.x;
    GS00 += b.y;
    GS11 += c.x;
    GS22 += c.y;
    GS01 += d.x;
    GS02 += d.y;
    GS12 += e.x;
    gop += e.y;
  }
  gp_tmp[4 * i] = gp0;
  gp_tmp[4 * i + 1] = gp1;
  gp_tmp[4 * i + 2] = gp2;
  reinterpret_cast<uint64_t*>(gp_tmp)[4 * i + 3] = mask;
  const float qf0 = quats[4 * i], qf1 = quats[4 * i + 1], qf2 = quats[4 * i + 2], qf3 = quats[4 * i + 3];
  const float lf0 = log_scales[3 * i], lf1 = log_scales[3 * i + 1], lf2 = log_scales[3 * i + 2];
  const float logit = logits[i];
  double q[4] = {qf0, qf1, qf2, qf3};
  const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (qn > 0.0)
    for (int k = 0; k < 4; ++k) q[k] /= qn;
  const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
  const double R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                       2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                       2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
  double GR[9], gl[3];
  for (int j = 0; j < 3; ++j) {
    const double Rj0 = R[j], Rj1 = R[3 + j], Rj2 = R[6 + j];
    const double G0 = GS00 * Rj0 + GS01 * Rj1 + GS02 * Rj2;
    const double G1 = GS01 * Rj0 + GS11 * Rj1 + GS12 * Rj2;
    const double G2 = GS02 * Rj0 + GS12 * Rj1 + GS22 * Rj2;
    const double s2 = exp(2.0 * (double)(j == 0 ? lf0 : (j == 1 ? lf1 : lf2)));
    gl[j] = 2.0 * s2 * (Rj0 * G0 + Rj1 * G1 + Rj2 * G2);
    GR[j] = 2.0 * s2 * G0;
    GR[3 + j] = 2.0 * s2 * G1;
    GR[6 + j] = 2.0 * s2 * G2;
  }
  const double dw = GR[1] * (-2 * qz) + GR[2] * (2 * qy) + GR[3] * (2 * qz) + GR[5] * (-2 * qx) +
                    GR[6] * (-2 * qy) + GR[7] * (2 * qx);
  const double dx = GR[1] * (2 * qy) + GR[2] * (2 * qz) + GR[3] * (2 * qy) + GR[4] * (-4 * qx) +
                    GR[5] * (-2 * qw) + GR[6] * (2 * qz) + GR[7] * (2 * qw) + GR[8] * (-4 * qx);
  const double dy = GR[0] * (-4 * qy) + GR[1] * (2 * qx) + GR[2] * (2 * qw) + GR[3] * (2 * qx) +
                    GR[5] * (2 * qz) + GR[6] * (-2 * qw) + GR[7] * (2 * qz) + GR[8] * (-4 * qy);
  const double dz = GR[0] * (-4 * qz) + GR[1] * (-2 * qw) + GR[2] * (2 * qx) + GR[3] * (2 * qw) +
                    GR[4] * (-4 * qz) + GR[5] * (2 * qy) + GR[6] * (2 * qx) + GR[7] * (2 * qy);
  const double dot = dw * qw + dx * qx + dy * qy + dz * qz;
  const double o = 1.0 / (1.0 + exp(-(double)logit));
  auto put = [&](float* dst, double val) { *dst = accumulate ? *dst + (float)val : (float)val; };
  for (int r = 0; r < 3; ++r) put(&g_ls[3 * i + r], gl[r]);
  const double qnn = qn > 0.0 ? qn : 1.0;
  put(&g_q[4 * i], (dw - dot * qw) / qnn);
  put(&g_q[4 * i + 1], (dx - dot * qx) / qnn);
  put(&g_q[4 * i + 2], (dy - dot * qy) / qnn);
  put(&g_q[4 * i + 3], (dz - dot * qz) / qnn);
  put(&g_logit[i], gop * o * (1.0 - o));
}

// Colour half per Gaussian: each view's colour chain (SH coefficients in
// LDS, their gradient sums in registers) in view order; the mean gradient
// is the projection half's sum plus the colour sum.
template <int DEG>
__global__ void __launch_bounds__(kGaussThreads) k_project_colour(
    const float* __restrict__ means, const float* __restrict__ sh, int64_t n,
    const float* __restrict__ cams, const double* __restrict__ terms, int accumulate,
    const double* __restrict__ gp_tmp, float* __restrict__ g_means, float* __restrict__ g_sh) {
  constexpr int K = (DEG + 1) * (DEG + 1), K3 = 3 * K;
  const int64_t i = (int64_t)blockIdx.x * kGaussThreads + threadIdx.x;
  if (i >= n) return;
  const uint64_t mask = reinterpret_cast<const uint64_t*>(gp_tmp)[4 * i + 3];
  __shared__ float s_shv[kGaussThreads][K3 + 1];
  float* shv = s_shv[threadIdx.x];
  float acc_sh[K3];
#pragma unroll
  for (int k = 0; k < K3; ++k) {
    shv[k] = sh[i * K3 + k];
    acc_sh[k] = 0.0f;
  }
  const double p[3] = {(double)means[3 * i], (double)means[3 * i + 1], (double)means[3 * i + 2]};
  double gc0 = 0, gc1 = 0, gc2 = 0;
  for (uint64_t m = mask; m; m &= m - 1) {
    const int v = __builtin_ctzll(m);
    const double2* src = reinterpret_cast<const double2*>(terms + ((int64_t)v * n + i) * kTermWords);
    const double2 a = src[5], b = src[6];
    const float* c = cams + (int64_t)v * GS_CAMERA_FLOATS;
    double W[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) W[e] = c[4 + e];
    const double g2c[3] = {a.x, a.y, b.x};
    double gv0, gv1, gv2;
    colour_term<DEG>(W, c[13], c[14], c[15], p, (uint32_t)b.y, g2c, shv, acc_sh, gv0, gv1, gv2);
    gc0 += W[0] * 0.0 + W[3] * 0.0 + W[6] * 0.0 + gv0;
    gc1 += W[1] * 0.0 + W[4] * 0.0 + W[7] * 0.0 + gv1;
    gc2 += W[2] * 0.0 + W[5] * 0.0 + W[8] * 0.0 + gv2;
  }
  float* gdst = g_sh + i * K3;
  if (accumulate) {
#pragma unroll
    for (int e = 0; e < K3; ++e) gdst[e] = gdst[e] + acc_sh[e];
  } else {
#pragma unroll
    for (int e = 0; e < K3; ++e) gdst[e] = acc_sh[e];
  }
  const double gp0 = gp_tmp[4 * i] + gc0, gp1 = gp_tmp[4 * i + 1] + gc1,
               gp2 = gp_tmp[4 * i + 2] + gc2;
  auto put = [&](float* dst, double val) { *dst = accumulate ? *dst + (float)val : (float)val; };
  put(&g_means[3 * i], gp0);
  put(&g_means[3 * i + 1], gp1);
  put(&g_means[3 * i + 2], gp2);
}

// Zero of the five gradient arrays (59 floats per Gaussian at degree 3).
__global__ void __launch_bounds__(256) k_zero_grads(float* __restrict__ a, int64_t na,
                                                    float* __restrict__ b, int64_t nb,
                                                    float* __restrict__ c, int64_t nc,
                                                    float* __restrict__ d, int64_t nd,
                                                    float* __restrict__ e, int64_t ne) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < na + nb + nc + nd + ne;
       k += stride) {
    int64_t r = k;
    if (r < na) { a[r] = 0.0f; continue; }
    r -= na;
    if (r < nb) { b[r] = 0.0f; continue; }
    r -= nb;
    if (r < nc) { c[r] = 0.0f; continue; }
    r -= nc;
    if (r < nd) { d[r] = 0.0f; continue; }
    r -= nd;
    e[r] = 0.0f;
  }
}

// Per-view camera tangent from the workgroup partials, fixed order.
__global__ void __launch_bounds__(256) k_pose_reduce(const double* __restrict__ pose_part,
                                                     int64_t nblocks, float* __restrict__ out) {
  const int v = blockIdx.x;
  __shared__ double red[256 / kWave][6];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nblocks; b += 256)
    for (int k = 0; k < 6; ++k) acc[k] += pose_part[((int64_t)v * nblocks + b) * 6 + k];
  for (int k = 0; k < 6; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane_id() == 0) red[threadIdx.x / kWave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int w = 0; w < 256 / kWave; ++w) s += red[w][threadIdx.x];
    out[6 * v + threadIdx.x] = (float)s;
  }
}

}  // namespace

// With one view the projection backward runs over the visible Gaussians
// only, so the others' gradients must be zeroed first (unless accumulating).
bool project_bwd_zeroes(const Plan& P, int accumulate) {
  return P.vt.n_views == 1 && !accumulate && P.n > 0;
}

hipError_t launch_zero_grads(const Plan& P, const gs_gaussian_grads& out, hipStream_t s) {
  const int64_t K3 = 3 * (int64_t)P.K;
  hipLaunchKernelGGL(k_zero_grads, dim3(2048), dim3(256), 0, s, out.means, 3 * P.n,
                     out.log_scales, 3 * P.n, out.quats, 4 * P.n, out.opacity_logits, P.n,
                     out.sh, K3 * P.n);
  return hipGetLastError();
}

// zeroed: the caller has already zeroed the gradients (see project_bwd_zeroes).
hipError_t launch_project_bwd(const Plan& P, const gs_gaussians& g, const float* cams, void* ws,
                              const gs_gaussian_grads& out, float* dL_dpose, int accumulate,
                              bool zeroed, hipStream_t s) {
  const int64_t blocks = P.proj_blocks;
  if (blocks == 0) return hipSuccess;
  // SPLIT workgroups (no camera tangent) take 64 Gaussians each
  const int64_t split_blocks = (P.n + kWave - 1) / kWave;
  double* pose_part = dL_dpose ? ws_at<double>(ws, P.off_pose_part) : nullptr;
  const bool compact = P.vt.n_views == 1;
  // several views without a camera tangent: a thread per visible record
  // (grid for all records; the count is on the device), then per Gaussian
  const int64_t rec_blocks = (P.n_rec + kRecThreads - 1) / kRecThreads;
  const int64_t gauss_blocks = (P.n + kGaussThreads - 1) / kGaussThreads;
  if (project_bwd_zeroes(P, accumulate) && !zeroed) {
    const hipError_t e = launch_zero_grads(P, out, s);
    if (e != hipSuccess) return e;
  }
#define GS_PB1(D, PO, CO)                                                                         \
  hipLaunchKernelGGL((k_project_bwd<D, PO, CO, !PO>), dim3((unsigned)(PO ? blocks : split_blocks)), \
                     dim3((CO && !PO) ? kSumWaves * kWave : kProjThreads), 0, s,                    \
                     g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, P.n, cams, P.vt,      \
                     ws_at<Rec>(ws, P.off_rec), ws_at<uint32_t>(ws, P.off_tt),                    \
                     ws_at<uint32_t>(ws, P.off_poff),                                              \
                     ws_at<float>(ws, P.off_grad_pair), ws_at<int32_t>(ws, P.off_flags),          \
                     ws_at<uint32_t>(ws, P.off_vis_list), accumulate, out.means, out.log_scales,  \
                     out.quats, out.opacity_logits, out.sh, pose_part, blocks)
// (one statement: the three launches of the several-view form)
#define GS_PBMV(D)                                                                                \
  do {                                                                                            \
    hipLaunchKernelGGL((k_project_rec<D>), dim3((unsigned)rec_blocks), dim3(kRecThreads), 0, s,    \
                       g.means, g.log_scales, g.quats, P.n, cams, P.vt,                           \
                       ws_at<uint32_t>(ws, P.off_tt), ws_at<uint32_t>(ws, P.off_poff),             \
                       ws_at<float>(ws, P.off_grad_pair), ws_at<int32_t>(ws, P.off_flags),         \
                       ws_at<uint32_t>(ws, P.off_vis_list), ws_at<uint32_t>(ws, P.off_vis_clamp),  \
                       ws_at<double>(ws, P.off_rec_terms));                                        \
    hipLaunchKernelGGL(k_project_gauss, dim3((unsigned)gauss_blocks), dim3(kGaussThreads), 0, s,   \
                       g.log_scales, g.quats, g.opacity_logits, P.n, P.vt.n_views,                  \
                       ws_at<uint32_t>(ws, P.off_tt), ws_at<double>(ws, P.off_rec_terms),          \
                       ws_at<int32_t>(ws, P.off_flags), accumulate,                                 \
                       ws_at<double>(ws, P.off_gp_tmp), out.log_scales, out.quats,                  \
                       out.opacity_logits);                                                         \
    hipLaunchKernelGGL((k_project_colour<D>), dim3((unsigned)gauss_blocks), dim3(kGaussThreads),   \
                       0, s, g.means, g.sh, P.n, cams, ws_at<double>(ws, P.off_rec_terms),         \
                       accumulate, ws_at<double>(ws, P.off_gp_tmp), out.means, out.sh);             \
  } while (0)
#define GS_PB(D)                \
  if (pose_part) {              \
    if (compact)                \
      GS_PB1(D, true, true);    \
    else                        \
      GS_PB1(D, true, false);   \
  } else {                      \
    if (compact)                \
      GS_PB1(D, false, true);   \
    else                        \
      GS_PBMV(D);               \
  }
  // the several-view form writes per-record slots and per-Gaussian sums that
  // only plans of several views allocate
  if (!pose_part && !compact && P.vt.n_views < 2) return hipErrorInvalidValue;
  switch (P.deg) {
    case 0: GS_PB(0); break;
    case 1: GS_PB(1); break;
    case 2: GS_PB(2); break;
    default: GS_PB(3); break;
  }
#undef GS_PB
#undef GS_PBMV
#undef GS_PB1
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dL_dpose) {
    hipLaunchKernelGGL(k_pose_reduce, dim3(P.vt.n_views), dim3(256), 0, s, pose_part, blocks,
                       dL_dpose);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace gs

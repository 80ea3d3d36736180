// a6: from per-pair 2D gradients to parameter and camera gradients.  One
// thread per Gaussian loops over the views: it sums the partials of its own
// (view, tile) pairs -- contiguous in generation order -- in a fixed order,
// recomputes the view's projection in FP64 and applies the chain rule
// through conic -> EWA covariance -> Jacobian -> camera-space mean, the 3D
// covariance (scale, rotation), the SH colour and the view direction, and
// the opacity sigmoid.  Camera tangents (rho, phi) for a left perturbation of
// each pose are reduced per workgroup (fixed order) and then per view.
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

// Real SH basis (orthonormal, Condon-Shortley phase) at unit direction (x,y,z).
template <int DEG>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double* Y) {
  Y[0] = kSH0;
  if (DEG >= 1) { Y[1] = -kSH1 * y; Y[2] = kSH1 * z; Y[3] = -kSH1 * x; }
  if (DEG >= 2) {
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2a * x * y;
    Y[5] = -kSH2a * y * z;
    Y[6] = kSH2b * (2 * zz - xx - yy);
    Y[7] = -kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = -kSH3a * y * (3 * xx - yy);
      Y[10] = kSH3b * x * y * z;
      Y[11] = -kSH3c * y * (4 * zz - xx - yy);
      Y[12] = kSH3d * z * (2 * zz - 3 * xx - 3 * yy);
      Y[13] = -kSH3c * x * (4 * zz - xx - yy);
      Y[14] = kSH3e * z * (xx - yy);
      Y[15] = -kSH3a * x * (xx - 3 * yy);
    }
  }
}

// g += sum_k w_k grad Y_k(x, y, z), the basis treated as polynomials in x,y,z.
template <int DEG>
__device__ __forceinline__ void sh_dir_grad(double x, double y, double z, const double* w,
                                            double& gx, double& gy, double& gz) {
  if (DEG >= 1) {
    gy += -kSH1 * w[1];
    gz += kSH1 * w[2];
    gx += -kSH1 * w[3];
  }
  if (DEG >= 2) {
    gx += kSH2a * y * w[4];           gy += kSH2a * x * w[4];
    gy += -kSH2a * z * w[5];          gz += -kSH2a * y * w[5];
    gx += -2 * kSH2b * x * w[6];      gy += -2 * kSH2b * y * w[6];  gz += 4 * kSH2b * z * w[6];
    gx += -kSH2a * z * w[7];          gz += -kSH2a * x * w[7];
    gx += 2 * kSH2c * x * w[8];       gy += -2 * kSH2c * y * w[8];
    if (DEG >= 3) {
      const double xx = x * x, yy = y * y, zz = z * z;
      gx += -6 * kSH3a * x * y * w[9];
      gy += -kSH3a * (3 * xx - 3 * yy) * w[9];
      gx += kSH3b * y * z * w[10];    gy += kSH3b * x * z * w[10];  gz += kSH3b * x * y * w[10];
      gx += 2 * kSH3c * x * y * w[11];
      gy += -kSH3c * (4 * zz - xx - 3 * yy) * w[11];
      gz += -8 * kSH3c * y * z * w[11];
      gx += -6 * kSH3d * x * z * w[12];
      gy += -6 * kSH3d * y * z * w[12];
      gz += kSH3d * (6 * zz - 3 * xx - 3 * yy) * w[12];
      gx += -kSH3c * (4 * zz - 3 * xx - yy) * w[13];
      gy += 2 * kSH3c * x * y * w[13];
      gz += -8 * kSH3c * x * z * w[13];
      gx += 2 * kSH3e * x * z * w[14]; gy += -2 * kSH3e * y * z * w[14]; gz += kSH3e * (xx - yy) * w[14];
      gx += -kSH3a * (3 * xx - 3 * yy) * w[15];
      gy += 6 * kSH3a * x * y * w[15];
    }
  }
}

template <int DEG>
__global__ void __launch_bounds__(kProjThreads) k_project_bwd(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, const float* __restrict__ cams, ViewTable vt,
    const uint32_t* __restrict__ tt, const uint32_t* __restrict__ poff,
    const float* __restrict__ grad_pair, const int32_t* __restrict__ fl, int accumulate,
    float* __restrict__ g_means, float* __restrict__ g_ls, float* __restrict__ g_q,
    float* __restrict__ g_logit, float* __restrict__ g_sh, double* __restrict__ pose_part,
    int64_t pose_stride) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  constexpr int NW = kProjThreads / kWave;
  const int64_t i = (int64_t)blockIdx.x * kProjThreads + threadIdx.x;
  const bool valid = i < n;
  const bool overflow = fl[F_OVERFLOW] != 0;
  __shared__ double spose[NW][6];

  double gp[3] = {0, 0, 0}, gl[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gb = 0.0;
  bool sh_written = false;
  // parameters (read once)
  double p[3] = {0, 0, 0}, s[3] = {1, 1, 1}, q[4] = {1, 0, 0, 0}, qn = 1.0, o = 0.0;
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double S00 = 0, S01 = 0, S02 = 0, S11 = 0, S12 = 0, S22 = 0;
  if (valid) {
    p[0] = means[3 * i]; p[1] = means[3 * i + 1]; p[2] = means[3 * i + 2];
    for (int k = 0; k < 3; ++k) s[k] = exp((double)log_scales[3 * i + k]);
    for (int k = 0; k < 4; ++k) q[k] = quats[4 * i + k];
    qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (qn > 0.0)
      for (int k = 0; k < 4; ++k) q[k] /= qn;
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
    const double s0 = s[0] * s[0], s1 = s[1] * s[1], s2 = s[2] * s[2];
    S00 = R[0] * R[0] * s0 + R[1] * R[1] * s1 + R[2] * R[2] * s2;
    S01 = R[0] * R[3] * s0 + R[1] * R[4] * s1 + R[2] * R[5] * s2;
    S02 = R[0] * R[6] * s0 + R[1] * R[7] * s1 + R[2] * R[8] * s2;
    S11 = R[3] * R[3] * s0 + R[4] * R[4] * s1 + R[5] * R[5] * s2;
    S12 = R[3] * R[6] * s0 + R[4] * R[7] * s1 + R[5] * R[8] * s2;
    S22 = R[6] * R[6] * s0 + R[7] * R[7] * s1 + R[8] * R[8] * s2;
    o = 1.0 / (1.0 + exp(-(double)logits[i]));
  }

  for (int v = 0; v < vt.n_views; ++v) {
    const int64_t ri = (int64_t)v * n + i;
    const uint32_t cnt = (valid && !overflow) ? tt[ri] : 0u;
    double pose[6] = {0, 0, 0, 0, 0, 0};
    if (cnt > 0) {
      // fixed-order sum of this (view, Gaussian)'s pair partials
      double g2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      const float4* gpp = reinterpret_cast<const float4*>(grad_pair + (int64_t)poff[ri] * kPairGrad);
      for (uint32_t k = 0; k < cnt; ++k) {
        const float4 a = gpp[3 * k], b = gpp[3 * k + 1], c = gpp[3 * k + 2];
        g2[0] += a.x; g2[1] += a.y; g2[2] += a.z; g2[3] += a.w;
        g2[4] += b.x; g2[5] += b.y; g2[6] += b.z; g2[7] += b.w;
        g2[8] += c.x; g2[9] += c.y;
      }
      const double g_rgb[3] = {g2[0], g2[1], g2[2]};
      const double g_depth = g2[3], g_op = g2[4];
      const double ga = g2[5], gbb = g2[6], gc = g2[7], gmx = g2[8], gmy = g2[9];

      const float* c = cams + (int64_t)v * GS_CAMERA_FLOATS;
      const double fx = c[0], fy = c[1];
      double W[9];
      for (int k = 0; k < 9; ++k) W[k] = c[4 + k];
      const double t0 = c[13], t1 = c[14], t2 = c[15];
      const double tx = W[0] * p[0] + W[1] * p[1] + W[2] * p[2] + t0;
      const double ty = W[3] * p[0] + W[4] * p[1] + W[5] * p[2] + t1;
      const double tz = W[6] * p[0] + W[7] * p[1] + W[8] * p[2] + t2;
      const double limx = 1.3 * (double)vt.v[v].W / (2.0 * fx);
      const double limy = 1.3 * (double)vt.v[v].H / (2.0 * fy);
      const double ux = tx / tz, vy = ty / tz;
      const bool cu = (ux < -limx) || (ux > limx), cv = (vy < -limy) || (vy > limy);
      const double u = fmin(limx, fmax(-limx, ux)), w = fmin(limy, fmax(-limy, vy));
      const double j00 = fx / tz, j02 = -fx * u / tz, j11 = fy / tz, j12 = -fy * w / tz;
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
      const double M00 = ya * ga + yb * 0.5 * gbb, M01 = ya * 0.5 * gbb + yb * gc;
      const double M10 = yb * ga + yc * 0.5 * gbb, M11 = yb * 0.5 * gbb + yc * gc;
      const double X00 = -(M00 * ya + M01 * yb), X01 = -(M00 * yb + M01 * yc),
                   X11 = -(M10 * yb + M11 * yc);
      // G_Sigma = X00 a a^T + X01 (a b^T + b a^T) + X11 b b^T
      const double av[3] = {a0, a1, a2}, bv[3] = {b0, b1, b2};
      double GS[3][3];
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
          GS[r][cc] = X00 * av[r] * av[cc] + X01 * (av[r] * bv[cc] + bv[r] * av[cc]) + X11 * bv[r] * bv[cc];
      // G_T2 rows: 2 (X00 Sa + X01 Sb), 2 (X01 Sa + X11 Sb);  G_J = G_T2 W^T
      const double gr0[3] = {2 * (X00 * Sa0 + X01 * Sb0), 2 * (X00 * Sa1 + X01 * Sb1), 2 * (X00 * Sa2 + X01 * Sb2)};
      const double gr1[3] = {2 * (X01 * Sa0 + X11 * Sb0), 2 * (X01 * Sa1 + X11 * Sb1), 2 * (X01 * Sa2 + X11 * Sb2)};
      const double GJ00 = gr0[0] * W[0] + gr0[1] * W[1] + gr0[2] * W[2];
      const double GJ02 = gr0[0] * W[6] + gr0[1] * W[7] + gr0[2] * W[8];
      const double GJ11 = gr1[0] * W[3] + gr1[1] * W[4] + gr1[2] * W[5];
      const double GJ12 = gr1[0] * W[6] + gr1[1] * W[7] + gr1[2] * W[8];
      const double tz2 = tz * tz, tz3 = tz2 * tz;
      double gt[3] = {0, 0, 0};
      gt[2] += -GJ00 * fx / tz2 - GJ11 * fy / tz2;
      if (!cu) { gt[0] += -GJ02 * fx / tz2; gt[2] += GJ02 * 2.0 * fx * tx / tz3; }
      else { gt[2] += GJ02 * fx * u / tz2; }
      if (!cv) { gt[1] += -GJ12 * fy / tz2; gt[2] += GJ12 * 2.0 * fy * ty / tz3; }
      else { gt[2] += GJ12 * fy * w / tz2; }
      gt[0] += gmx * fx / tz;
      gt[1] += gmy * fy / tz;
      gt[2] += -(gmx * fx * tx + gmy * fy * ty) / tz2 + g_depth;

      // colour: SH coefficients and view direction
      const double cxw = -(W[0] * t0 + W[3] * t1 + W[6] * t2);
      const double cyw = -(W[1] * t0 + W[4] * t1 + W[7] * t2);
      const double czw = -(W[2] * t0 + W[5] * t1 + W[8] * t2);
      const double dv0 = p[0] - cxw, dv1 = p[1] - cyw, dv2 = p[2] - czw;
      const double dist = sqrt(dv0 * dv0 + dv1 * dv1 + dv2 * dv2);
      const double d0 = dv0 / dist, d1 = dv1 / dist, d2 = dv2 / dist;
      double Y[16];
      sh_basis<DEG>(d0, d1, d2, Y);
      const float* shp = sh + i * (K * 3);
      float* gsh = g_sh + i * (K * 3);
      double raw[3] = {0.5, 0.5, 0.5};
      for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) raw[ch] += (double)shp[3 * k + ch] * Y[k];
      double gcr[3];
      for (int ch = 0; ch < 3; ++ch) gcr[ch] = raw[ch] < 0.0 ? 0.0 : g_rgb[ch];
      // per-basis weights w_k = sum_ch gcr_ch SH_k,ch and the SH gradients
      double wk[16];
      const bool first = !sh_written && !accumulate;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        wk[k] = 0.0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          wk[k] += gcr[ch] * (double)shp[3 * k + ch];
          const float add = (float)(Y[k] * gcr[ch]);
          gsh[3 * k + ch] = first ? add : gsh[3 * k + ch] + add;
        }
      }
      double gd[3] = {0, 0, 0};
      sh_dir_grad<DEG>(d0, d1, d2, wk, gd[0], gd[1], gd[2]);
      sh_written = true;
      const double dd = gd[0] * d0 + gd[1] * d1 + gd[2] * d2;
      const double gv[3] = {(gd[0] - dd * d0) / dist, (gd[1] - dd * d1) / dist, (gd[2] - dd * d2) / dist};
      // mean
      for (int r = 0; r < 3; ++r) gp[r] += W[r] * gt[0] + W[3 + r] * gt[1] + W[6 + r] * gt[2] + gv[r];
      // scale and rotation: G_R[:, j] = 2 s_j^2 G_Sigma R_j ; g_l_j = s_j^2 * 2 R_j^T G_Sigma R_j
      double GR[9];
      for (int j = 0; j < 3; ++j) {
        const double Rj[3] = {R[j], R[3 + j], R[6 + j]};
        const double GRj[3] = {GS[0][0] * Rj[0] + GS[0][1] * Rj[1] + GS[0][2] * Rj[2],
                               GS[1][0] * Rj[0] + GS[1][1] * Rj[1] + GS[1][2] * Rj[2],
                               GS[2][0] * Rj[0] + GS[2][1] * Rj[1] + GS[2][2] * Rj[2]};
        const double s2 = s[j] * s[j];
        gl[j] += 2.0 * s2 * (Rj[0] * GRj[0] + Rj[1] * GRj[1] + Rj[2] * GRj[2]);
        GR[j] = 2.0 * s2 * GRj[0];
        GR[3 + j] = 2.0 * s2 * GRj[1];
        GR[6 + j] = 2.0 * s2 * GRj[2];
      }
      {
        const double qw = q[0], qx = q[1], qy = q[2], qz = q[3];
        const double dw = GR[1] * (-2 * qz) + GR[2] * (2 * qy) + GR[3] * (2 * qz) + GR[5] * (-2 * qx) +
                          GR[6] * (-2 * qy) + GR[7] * (2 * qx);
        const double dx = GR[1] * (2 * qy) + GR[2] * (2 * qz) + GR[3] * (2 * qy) + GR[4] * (-4 * qx) +
                          GR[5] * (-2 * qw) + GR[6] * (2 * qz) + GR[7] * (2 * qw) + GR[8] * (-4 * qx);
        const double dy = GR[0] * (-4 * qy) + GR[1] * (2 * qx) + GR[2] * (2 * qw) + GR[3] * (2 * qx) +
                          GR[5] * (2 * qz) + GR[6] * (-2 * qw) + GR[7] * (2 * qz) + GR[8] * (-4 * qy);
        const double dz = GR[0] * (-4 * qz) + GR[1] * (-2 * qw) + GR[2] * (2 * qx) + GR[3] * (2 * qw) +
                          GR[4] * (-4 * qz) + GR[5] * (2 * qy) + GR[6] * (2 * qx) + GR[7] * (2 * qy);
        const double dot = dw * qw + dx * qx + dy * qy + dz * qz;
        gq[0] += (dw - dot * qw) / qn;
        gq[1] += (dx - dot * qx) / qn;
        gq[2] += (dy - dot * qy) / qn;
        gq[3] += (dz - dot * qz) / qn;
      }
      gb += g_op * o * (1.0 - o);
      // camera tangent
      for (int r = 0; r < 3; ++r) pose[r] = gt[r] + W[3 * r] * gv[0] + W[3 * r + 1] * gv[1] + W[3 * r + 2] * gv[2];
      pose[3] = ty * gt[2] - tz * gt[1];
      pose[4] = tz * gt[0] - tx * gt[2];
      pose[5] = tx * gt[1] - ty * gt[0];
      // Sigma_c = W Sigma W^T ;  G_c = J^T X J (J has j01 = j10 = 0)
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
      // A = Sc Gc - Gc Sc ; g_phi -= 2 (A21, A02, A10)
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
    if (pose_part) {
      // workgroup sum of the camera tangent for this view, fixed order
      const int w = threadIdx.x / kWave;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double sum = wave_sum(pose[k]);
        if (lane_id() == 0) spose[w][k] = sum;
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
  if (!valid) return;
  auto put = [&](float* dst, double val) { *dst = accumulate ? *dst + (float)val : (float)val; };
  for (int r = 0; r < 3; ++r) put(&g_means[3 * i + r], gp[r]);
  for (int r = 0; r < 3; ++r) put(&g_ls[3 * i + r], gl[r]);
  for (int r = 0; r < 4; ++r) put(&g_q[4 * i + r], gq[r]);
  put(&g_logit[i], gb);
  if (!sh_written && !accumulate) {
    float* gsh = g_sh + i * (K * 3);
    for (int k = 0; k < K * 3; ++k) gsh[k] = 0.0f;
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

hipError_t launch_project_bwd(const Plan& P, const gs_gaussians& g, const float* cams, void* ws,
                              const gs_gaussian_grads& out, float* dL_dpose, int accumulate,
                              hipStream_t s) {
  const int64_t blocks = P.proj_blocks;
  if (blocks == 0) return hipSuccess;
  double* pose_part = dL_dpose ? ws_at<double>(ws, P.off_pose_part) : nullptr;
#define GS_PB(D)                                                                              \
  hipLaunchKernelGGL(k_project_bwd<D>, dim3((unsigned)blocks), dim3(kProjThreads), 0, s,       \
                     g.means, g.log_scales, g.quats, g.opacity_logits, g.sh, P.n, cams, P.vt,  \
                     ws_at<uint32_t>(ws, P.off_tt), ws_at<uint32_t>(ws, P.off_poff),          \
                     ws_at<float>(ws, P.off_grad_pair), ws_at<int32_t>(ws, P.off_flags),      \
                     accumulate, out.means, out.log_scales, out.quats, out.opacity_logits,    \
                     out.sh, pose_part, blocks)
  switch (P.deg) {
    case 0: GS_PB(0); break;
    case 1: GS_PB(1); break;
    case 2: GS_PB(2); break;
    default: GS_PB(3); break;
  }
#undef GS_PB
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

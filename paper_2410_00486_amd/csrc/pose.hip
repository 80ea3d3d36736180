// Camera-pose tangent of the differentiable render (the camera gradient that
// SLAM back-ends optimise beside the map).  The renderer's camera gradient
// is taken with respect to a left perturbation delta = (rho, phi) of the
// world->camera pose, evaluated at zero:
//     R <- Exp(phi) R,   t <- Exp(phi) t + rho.
// A caller that optimises a tangent xi applies the same map at xi
// (gs_pose_retract) and needs dL/dxi.  Away from zero the two differ:
// Exp(phi + dphi) = Exp(J(phi) dphi) Exp(phi) with J the left Jacobian of
// SO(3), and the translation picks up rho x (J dphi), so
//     dL/drho = g_rho,    dL/dphi = J^T (g_phi - rho x g_rho)
// with (g_rho, g_phi) = dL/ddelta at the retracted pose (gs_pose_tangent_vjp).
// One thread per view, FP64 throughout, results rounded once to float32.
#include "gs_internal.h"

namespace gs {
namespace {

// Coefficients of the SO(3) series in theta = |phi|:
//   a = sin(th)/th, b = (1 - cos th)/th^2, c = (th - sin th)/th^3,
// so that Exp(phi) = I + a [phi]x + b [phi]x^2 and J(phi) = I + b [phi]x +
// c [phi]x^2.  Below th = 1e-2 the Taylor series to th^4 (next terms below
// 3e-16) replaces the quotients, whose cancellation grows as th -> 0.
__device__ void so3_coeffs(const double phi[3], double& a, double& b, double& c) {
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  if (th2 < 1e-4) {
    a = 1.0 - th2 / 6.0 * (1.0 - th2 / 20.0);
    b = 0.5 - th2 / 24.0 * (1.0 - th2 / 30.0);
    c = 1.0 / 6.0 - th2 / 120.0 * (1.0 - th2 / 42.0);
  } else {
    const double th = sqrt(th2);
    const double s = sin(th), co = cos(th);
    a = s / th;
    b = (1.0 - co) / th2;
    c = (th - s) / (th2 * th);
  }
}

// M = I + p [phi]x + q [phi]x^2, row-major.
__device__ void so3_poly(const double phi[3], double p, double q, double M[9]) {
  const double x = phi[0], y = phi[1], z = phi[2];
  // [phi]x = [[0, -z, y], [z, 0, -x], [-y, x, 0]]
  const double K[9] = {0.0, -z, y, z, 0.0, -x, -y, x, 0.0};
  // [phi]x^2 = phi phi^T - |phi|^2 I
  const double n2 = x * x + y * y + z * z;
  const double K2[9] = {x * x - n2, x * y, x * z, y * x, y * y - n2, y * z, z * x, z * y, z * z - n2};
  for (int k = 0; k < 9; ++k) M[k] = (k % 4 == 0 ? 1.0 : 0.0) + p * K[k] + q * K2[k];
}

__global__ void k_pose_retract(const float* __restrict__ cams_in, const float* __restrict__ xi,
                               float* __restrict__ cams_out, int n_views) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_views) return;
  const float* c = cams_in + (size_t)v * GS_CAMERA_FLOATS;
  float* o = cams_out + (size_t)v * GS_CAMERA_FLOATS;
  const double rho[3] = {xi[6 * v], xi[6 * v + 1], xi[6 * v + 2]};
  const double phi[3] = {xi[6 * v + 3], xi[6 * v + 4], xi[6 * v + 5]};
  double a, b, cc, E[9];
  so3_coeffs(phi, a, b, cc);
  so3_poly(phi, a, b, E);
  // record: fx fy cx cy | R[9] | t[3] | near | bg[3]
  double R[9], t[3];
  for (int k = 0; k < 9; ++k) R[k] = c[4 + k];
  for (int k = 0; k < 3; ++k) t[k] = c[13 + k];
  float out[GS_CAMERA_FLOATS];
  for (int k = 0; k < GS_CAMERA_FLOATS; ++k) out[k] = c[k];
  for (int r = 0; r < 3; ++r) {
    for (int col = 0; col < 3; ++col)
      out[4 + 3 * r + col] =
          (float)(E[3 * r] * R[col] + E[3 * r + 1] * R[3 + col] + E[3 * r + 2] * R[6 + col]);
    out[13 + r] = (float)(E[3 * r] * t[0] + E[3 * r + 1] * t[1] + E[3 * r + 2] * t[2] + rho[r]);
  }
  for (int k = 0; k < GS_CAMERA_FLOATS; ++k) o[k] = out[k];
}

__global__ void k_pose_vjp(const float* __restrict__ xi, const float* __restrict__ g_delta,
                           float* __restrict__ g_xi, int n_views) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_views) return;
  const double rho[3] = {xi[6 * v], xi[6 * v + 1], xi[6 * v + 2]};
  const double phi[3] = {xi[6 * v + 3], xi[6 * v + 4], xi[6 * v + 5]};
  const double gr[3] = {g_delta[6 * v], g_delta[6 * v + 1], g_delta[6 * v + 2]};
  const double gp[3] = {g_delta[6 * v + 3], g_delta[6 * v + 4], g_delta[6 * v + 5]};
  double a, b, c, J[9];
  so3_coeffs(phi, a, b, c);
  so3_poly(phi, b, c, J);
  // u = g_phi - rho x g_rho;  dL/dphi = J^T u
  const double u[3] = {gp[0] - (rho[1] * gr[2] - rho[2] * gr[1]),
                       gp[1] - (rho[2] * gr[0] - rho[0] * gr[2]),
                       gp[2] - (rho[0] * gr[1] - rho[1] * gr[0])};
  float out[6];
  for (int k = 0; k < 3; ++k) {
    out[k] = (float)gr[k];
    out[3 + k] = (float)(J[k] * u[0] + J[3 + k] * u[1] + J[6 + k] * u[2]);
  }
  for (int k = 0; k < 6; ++k) g_xi[6 * v + k] = out[k];
}

}  // namespace

hipError_t launch_pose_retract(const float* cams_in, const float* xi, float* cams_out,
                               int n_views, hipStream_t s) {
  hipLaunchKernelGGL(k_pose_retract, dim3((n_views + 63) / 64), dim3(64), 0, s, cams_in, xi,
                     cams_out, n_views);
  return hipGetLastError();
}

hipError_t launch_pose_vjp(const float* xi, const float* g_delta, float* g_xi, int n_views,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_pose_vjp, dim3((n_views + 63) / 64), dim3(64), 0, s, xi, g_delta, g_xi,
                     n_views);
  return hipGetLastError();
}

}  // namespace gs

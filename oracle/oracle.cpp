// FP64 CPU oracle for the differentiable 3D Gaussian-splatting rasterizer
// (CaRtGS, Sec. III-B Eq. (1) forward; Sec. III-C-1 Eqs. (2)-(4) backward).
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It is a plain, slow,
// obviously-correct reference: every quantity is computed in double
// precision with straightforward loops, one pixel / one Gaussian at a time.
// It shares no code, header, constant table or helper with the GPU library.
//
// Readings of the paper that this file follows (the paper retains the 3DGS
// conventions, Sec. IV-A "Implementation Detail"):
//   * Eq. (1) composites front to back, C = sum_k c_k a_k prod_{j<k}(1-a_j)
//     (the product index in the printed equation is read as j), plus the
//     background times the final transmittance.
//   * a_k = min(0.99, o_k G_k(pixel)); a Gaussian is skipped when its
//     Gaussian exponent is positive or when a_k < 1/255; blending stops
//     (without blending the current Gaussian) when T (1 - a_k) < 1e-4.
//   * EWA splatting with a 0.3 px^2 dilation, the Jacobian evaluated at a
//     camera-space point whose x/z, y/z are clamped to 1.3 x the half field
//     of view, Gaussians culled at z <= near.  These constants are
//     conventions: parity unpinned as values (the tests pin the formulas).
//   * Tile membership is the exact axis-aligned box of the a >= 1/255
//     ellipse, half extents kappa*sqrt(Sigma'_xx), kappa*sqrt(Sigma'_yy) with
//     kappa^2 = 2 ln(255 o), widened by a relative 1e-4 plus 1e-3 px.
//   * Depth ordering uses the float32 rounding of camera-space z, ties broken
//     by Gaussian index.
//   * The backward pass (Eqs. (2)-(4)) is the exact reverse-mode derivative
//     of the piecewise-smooth forward map with all discrete decisions fixed.
//   * The camera gradient is taken for a left perturbation of the
//     world->camera pose, T <- Exp(xi) T with xi = (rho, phi), R' = Exp(phi)R,
//     t' = Exp(phi) t + rho, evaluated at xi = 0.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr double kAlphaMax = 0.99;
constexpr double kAlphaMin = 1.0 / 255.0;
constexpr double kTransmittanceMin = 1e-4;
constexpr double kDilation = 0.3;
constexpr double kFovClamp = 1.3;
constexpr double kRectRel = 1e-4;
constexpr double kRectAbs = 1e-3;
// Relative band around a discrete threshold inside which a pixel or
// Gaussian is reported as "near a decision" (excluded from strict parity).
constexpr double kBand = 1e-5;

struct Cam {
  double fx, fy, cx, cy;
  double R[9];
  double t[3];
  double near_z;
  double bg[3];
  int width, height;
};

Cam load_cam(const double* c, int width, int height) {
  Cam k;
  k.fx = c[0]; k.fy = c[1]; k.cx = c[2]; k.cy = c[3];
  for (int i = 0; i < 9; ++i) k.R[i] = c[4 + i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[13 + i];
  k.near_z = c[16];
  for (int i = 0; i < 3; ++i) k.bg[i] = c[17 + i];
  k.width = width; k.height = height;
  return k;
}

// ---------------------------------------------------------------------------
// real spherical harmonics up to degree 3 (orthonormal, Condon-Shortley phase)
// evaluated at a unit direction, and their gradients as polynomials in x,y,z.
// ---------------------------------------------------------------------------
void sh_basis(double x, double y, double z, double Y[16]) {
  const double pi = M_PI;
  const double c0 = 0.5 / std::sqrt(pi);
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  const double c2a = 0.5 * std::sqrt(15.0 / pi);
  const double c2b = 0.25 * std::sqrt(5.0 / pi);
  const double c2c = 0.25 * std::sqrt(15.0 / pi);
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));
  const double c3b = 0.5 * std::sqrt(105.0 / pi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));
  const double c3d = 0.25 * std::sqrt(7.0 / pi);
  const double c3e = 0.25 * std::sqrt(105.0 / pi);
  Y[0] = c0;
  Y[1] = -c1 * y;
  Y[2] = c1 * z;
  Y[3] = -c1 * x;
  Y[4] = c2a * x * y;
  Y[5] = -c2a * y * z;
  Y[6] = c2b * (2 * z * z - x * x - y * y);
  Y[7] = -c2a * x * z;
  Y[8] = c2c * (x * x - y * y);
  Y[9] = -c3a * y * (3 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = -c3c * y * (4 * z * z - x * x - y * y);
  Y[12] = c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
  Y[13] = -c3c * x * (4 * z * z - x * x - y * y);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = -c3a * x * (x * x - 3 * y * y);
}

// dY[k][0..2] = d Y_k / d(x, y, z)
void sh_basis_grad(double x, double y, double z, double dY[16][3]) {
  const double pi = M_PI;
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  const double c2a = 0.5 * std::sqrt(15.0 / pi);
  const double c2b = 0.25 * std::sqrt(5.0 / pi);
  const double c2c = 0.25 * std::sqrt(15.0 / pi);
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi));
  const double c3b = 0.5 * std::sqrt(105.0 / pi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi));
  const double c3d = 0.25 * std::sqrt(7.0 / pi);
  const double c3e = 0.25 * std::sqrt(105.0 / pi);
  auto set = [&](int k, double a, double b, double c) { dY[k][0] = a; dY[k][1] = b; dY[k][2] = c; };
  set(0, 0, 0, 0);
  set(1, 0, -c1, 0);
  set(2, 0, 0, c1);
  set(3, -c1, 0, 0);
  set(4, c2a * y, c2a * x, 0);
  set(5, 0, -c2a * z, -c2a * y);
  set(6, -2 * c2b * x, -2 * c2b * y, 4 * c2b * z);
  set(7, -c2a * z, 0, -c2a * x);
  set(8, 2 * c2c * x, -2 * c2c * y, 0);
  set(9, -c3a * 6 * x * y, -c3a * (3 * x * x - 3 * y * y), 0);
  set(10, c3b * y * z, c3b * x * z, c3b * x * y);
  set(11, c3c * 2 * x * y, -c3c * (4 * z * z - x * x - 3 * y * y), -c3c * 8 * y * z);
  set(12, -c3d * 6 * x * z, -c3d * 6 * y * z, c3d * (6 * z * z - 3 * x * x - 3 * y * y));
  set(13, -c3c * (4 * z * z - 3 * x * x - y * y), c3c * 2 * x * y, -c3c * 8 * x * z);
  set(14, c3e * 2 * x * z, -c3e * 2 * y * z, c3e * (x * x - y * y));
  set(15, -c3a * (3 * x * x - 3 * y * y), c3a * 6 * x * y, 0);
}

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
void quat_to_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// dR/dq_k for k = w, x, y, z (row-major 3x3 each), for the formula above.
void quat_to_rot_grad(const double q[4], double dR[4][9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  const double Dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
  const double Dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
  const double Dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
  const double Dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
  std::memcpy(dR[0], Dw, sizeof Dw);
  std::memcpy(dR[1], Dx, sizeof Dx);
  std::memcpy(dR[2], Dy, sizeof Dy);
  std::memcpy(dR[3], Dz, sizeof Dz);
}

inline double sigmoid(double b) { return 1.0 / (1.0 + std::exp(-b)); }

// Everything the forward projection of one Gaussian in one view produces.
struct Proj {
  int status;            // 1 visible, 0 culled, 2 culled for non-finite input
  double q[4];           // normalised quaternion
  double qnorm;
  double s[3];           // scales
  double Rq[9];          // rotation of the Gaussian
  double Sigma[9];       // world covariance
  double tc[3];          // camera-space mean
  double u, v;           // clamped x/z, y/z
  bool clamp_u, clamp_v;
  double J[6];           // 2x3 Jacobian
  double T2[9];          // rows 0..1 used: J W (2x3)
  double cov[3];         // Sigma' = (A, B, C)
  double det;
  double conic[3];       // (a, b, c) = (C, -B, A) / det
  double mean2d[2];
  double opacity;
  double kappa;
  double dir[3];         // unit view direction from the camera centre
  double dist;           // |p - camera centre|
  double rgb_raw[3];
  double rgb[3];
  int rect[4];           // tile rect [x0, y0, x1, y1), clamped
  float depth32;
  int near_edge;         // rect edge or depth rounding within a tiny band
};

bool finite_all(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

void project_one(int64_t i, int deg, const double* means, const double* log_scales,
                 const double* quats, const double* logits, const double* sh,
                 const Cam& cam, int tw, int th, int cutoff_3sigma, Proj& P) {
  std::memset(&P, 0, sizeof P);
  const int K = (deg + 1) * (deg + 1);
  P.status = 0;
  if (!finite_all(means + 3 * i, 3) || !finite_all(log_scales + 3 * i, 3) ||
      !finite_all(quats + 4 * i, 4) || !finite_all(logits + i, 1) ||
      !finite_all(sh + (int64_t)K * 3 * i, K * 3)) {
    P.status = 2;
    return;
  }
  double q[4];
  for (int k = 0; k < 4; ++k) q[k] = quats[4 * i + k];
  const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if (!(qn > 0.0)) return;
  for (int k = 0; k < 4; ++k) P.q[k] = q[k] / qn;
  P.qnorm = qn;
  for (int k = 0; k < 3; ++k) P.s[k] = std::exp(log_scales[3 * i + k]);
  quat_to_rot(P.q, P.Rq);
  // Sigma = R diag(s^2) R^T
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += P.Rq[3 * r + k] * P.s[k] * P.s[k] * P.Rq[3 * c + k];
      P.Sigma[3 * r + c] = acc;
    }
  P.opacity = sigmoid(logits[i]);
  const double p[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  for (int r = 0; r < 3; ++r)
    P.tc[r] = cam.R[3 * r] * p[0] + cam.R[3 * r + 1] * p[1] + cam.R[3 * r + 2] * p[2] + cam.t[r];
  const double tx = P.tc[0], ty = P.tc[1], tz = P.tc[2];
  if (!(tz > cam.near_z)) return;
  P.mean2d[0] = cam.fx * tx / tz + cam.cx;
  P.mean2d[1] = cam.fy * ty / tz + cam.cy;
  const double limx = kFovClamp * cam.width / (2.0 * cam.fx);
  const double limy = kFovClamp * cam.height / (2.0 * cam.fy);
  const double ux = tx / tz, vy = ty / tz;
  P.u = std::min(limx, std::max(-limx, ux));
  P.v = std::min(limy, std::max(-limy, vy));
  P.clamp_u = (ux < -limx) || (ux > limx);
  P.clamp_v = (vy < -limy) || (vy > limy);
  P.J[0] = cam.fx / tz; P.J[1] = 0; P.J[2] = -cam.fx * P.u / tz;
  P.J[3] = 0; P.J[4] = cam.fy / tz; P.J[5] = -cam.fy * P.v / tz;
  // T2 = J W (2x3)
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += P.J[3 * r + k] * cam.R[3 * k + c];
      P.T2[3 * r + c] = acc;
    }
  // Sigma' = T2 Sigma T2^T + dilation I
  double S2[4];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      double acc = 0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc += P.T2[3 * r + a] * P.Sigma[3 * a + b] * P.T2[3 * c + b];
      S2[2 * r + c] = acc;
    }
  P.cov[0] = S2[0] + kDilation;
  P.cov[1] = 0.5 * (S2[1] + S2[2]);
  P.cov[2] = S2[3] + kDilation;
  P.det = P.cov[0] * P.cov[2] - P.cov[1] * P.cov[1];
  if (!(P.det > 0.0)) return;
  P.conic[0] = P.cov[2] / P.det;
  P.conic[1] = -P.cov[1] / P.det;
  P.conic[2] = P.cov[0] / P.det;
  if (P.opacity < kAlphaMin) return;
  P.kappa = std::sqrt(2.0 * std::log(255.0 * P.opacity));
  double hx, hy;
  if (cutoff_3sigma) {
    const double mid = 0.5 * (P.cov[0] + P.cov[2]);
    const double lmax = mid + std::sqrt(std::max(0.1, mid * mid - P.det));
    hx = hy = 3.0 * std::sqrt(lmax);
  } else {
    hx = P.kappa * std::sqrt(P.cov[0]);
    hy = P.kappa * std::sqrt(P.cov[2]);
  }
  hx = hx * (1.0 + kRectRel) + kRectAbs;
  hy = hy * (1.0 + kRectRel) + kRectAbs;
  const int tiles_x = (cam.width + tw - 1) / tw;
  const int tiles_y = (cam.height + th - 1) / th;
  auto tile_lo = [](double v, int ts, int nt) {
    double f = std::floor(v / ts);
    return (int)std::max(0.0, std::min((double)nt, f));
  };
  auto tile_hi = [](double v, int ts, int nt) {
    double f = std::floor(v / ts) + 1.0;
    return (int)std::max(0.0, std::min((double)nt, f));
  };
  P.rect[0] = tile_lo(P.mean2d[0] - hx, tw, tiles_x);
  P.rect[1] = tile_lo(P.mean2d[1] - hy, th, tiles_y);
  P.rect[2] = tile_hi(P.mean2d[0] + hx, tw, tiles_x);
  P.rect[3] = tile_hi(P.mean2d[1] + hy, th, tiles_y);
  if (P.rect[2] <= P.rect[0] || P.rect[3] <= P.rect[1]) return;
  // rect edges within a tiny band of a tile boundary, or a depth whose
  // float32 rounding is ambiguous: reported, not culled.
  auto near_int = [](double v) { return std::fabs(v - std::nearbyint(v)) < 1e-9 * std::max(1.0, std::fabs(v)); };
  P.near_edge = near_int((P.mean2d[0] - hx) / tw) || near_int((P.mean2d[0] + hx) / tw) ||
                near_int((P.mean2d[1] - hy) / th) || near_int((P.mean2d[1] + hy) / th);
  if ((float)(tz * (1 + 1e-13)) != (float)(tz * (1 - 1e-13))) P.near_edge = 1;
  P.depth32 = (float)tz;
  // view-dependent colour
  double cc[3];
  for (int r = 0; r < 3; ++r)
    cc[r] = -(cam.R[r] * cam.t[0] + cam.R[3 + r] * cam.t[1] + cam.R[6 + r] * cam.t[2]);
  double dv[3] = {p[0] - cc[0], p[1] - cc[1], p[2] - cc[2]};
  P.dist = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  for (int r = 0; r < 3; ++r) P.dir[r] = dv[r] / P.dist;
  double Y[16];
  sh_basis(P.dir[0], P.dir[1], P.dir[2], Y);
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0;
    for (int k = 0; k < K; ++k) acc += sh[((int64_t)i * K + k) * 3 + ch] * Y[k];
    P.rgb_raw[ch] = acc + 0.5;
    P.rgb[ch] = std::max(0.0, P.rgb_raw[ch]);
  }
  P.status = 1;
}

}  // namespace

extern "C" {

int ora_version() { return 4; }

// World-space covariance Sigma = R(q/|q|) diag(exp(2 l)) R^T of n Gaussians
// (row-major 3x3 each), exposed so tests can pin the rotation convention.
void ora_covariance3d(int64_t n, const double* log_scales, const double* quats, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    double q[4];
    double qn = 0;
    for (int k = 0; k < 4; ++k) { q[k] = quats[4 * i + k]; qn += q[k] * q[k]; }
    qn = std::sqrt(qn);
    for (int k = 0; k < 4; ++k) q[k] /= qn;
    double R[9];
    quat_to_rot(q, R);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k)
          acc += R[3 * r + k] * std::exp(2.0 * log_scales[3 * i + k]) * R[3 * c + k];
        out[9 * i + 3 * r + c] = acc;
      }
  }
}

// Per-Gaussian projection of one view (see project_one).  Outputs are
// arrays of length n (times the stated width); culled entries are zero.
void ora_preprocess(int64_t n, int deg, const double* means, const double* log_scales,
                    const double* quats, const double* logits, const double* sh,
                    const double* cam20, int width, int height, int tw, int th,
                    int cutoff_3sigma,
                    double* mean2d, double* conic, double* cov2d, double* opacity,
                    double* rgb, double* depth, float* depth32, int32_t* rect,
                    int32_t* tiles_touched, uint8_t* clamp_mask, int32_t* status,
                    int32_t* near_edge) {
  const Cam cam = load_cam(cam20, width, height);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Proj P;
    project_one(i, deg, means, log_scales, quats, logits, sh, cam, tw, th, cutoff_3sigma, P);
    const bool vis = P.status == 1;
    status[i] = P.status;
    mean2d[2 * i] = vis ? P.mean2d[0] : 0; mean2d[2 * i + 1] = vis ? P.mean2d[1] : 0;
    for (int k = 0; k < 3; ++k) {
      conic[3 * i + k] = vis ? P.conic[k] : 0;
      cov2d[3 * i + k] = vis ? P.cov[k] : 0;
      rgb[3 * i + k] = vis ? P.rgb[k] : 0;
    }
    opacity[i] = vis ? P.opacity : 0;
    depth[i] = vis ? P.tc[2] : 0;
    depth32[i] = vis ? P.depth32 : 0.0f;
    for (int k = 0; k < 4; ++k) rect[4 * i + k] = vis ? P.rect[k] : 0;
    tiles_touched[i] = vis ? (P.rect[2] - P.rect[0]) * (P.rect[3] - P.rect[1]) : 0;
    clamp_mask[i] = vis ? (uint8_t)((P.rgb_raw[0] < 0) | ((P.rgb_raw[1] < 0) << 1) |
                                    ((P.rgb_raw[2] < 0) << 2))
                        : 0;
    near_edge[i] = vis ? P.near_edge : 0;
  }
}

// Pair list of one view: keys (tile << 32 | float bits of depth) and values
// (Gaussian index), generated Gaussian by Gaussian, tiles in row-major rect
// order, then stably sorted by key.  Returns the pair count P; ranges gets
// [start, end) per tile.  keys/vals must hold sum(tiles_touched) entries.
int64_t ora_sort_pairs(int64_t n, const int32_t* rect, const int32_t* tiles_touched,
                       const float* depth32, int tiles_x, int n_tiles,
                       uint64_t* keys, uint32_t* vals, uint32_t* ranges) {
  int64_t P = 0;
  for (int64_t i = 0; i < n; ++i) P += tiles_touched[i];
  std::vector<uint64_t> k(P);
  std::vector<uint32_t> v(P);
  int64_t o = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (tiles_touched[i] == 0) continue;
    uint32_t dbits;
    std::memcpy(&dbits, &depth32[i], 4);
    for (int y = rect[4 * i + 1]; y < rect[4 * i + 3]; ++y)
      for (int x = rect[4 * i]; x < rect[4 * i + 2]; ++x) {
        const uint64_t tile = (uint64_t)(y * tiles_x + x);
        k[o] = (tile << 32) | dbits;
        v[o] = (uint32_t)i;
        ++o;
      }
  }
  std::vector<int64_t> idx(P);
  for (int64_t j = 0; j < P; ++j) idx[j] = j;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return k[a] < k[b]; });
  for (int64_t j = 0; j < P; ++j) {
    keys[j] = k[idx[j]];
    vals[j] = v[idx[j]];
  }
  for (int t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
  for (int64_t j = 0; j < P; ++j) {
    const uint32_t t = (uint32_t)(keys[j] >> 32);
    if (j == 0 || (uint32_t)(keys[j - 1] >> 32) != t) ranges[2 * t] = (uint32_t)j;
    if (j == P - 1 || (uint32_t)(keys[j + 1] >> 32) != t) ranges[2 * t + 1] = (uint32_t)(j + 1);
  }
  return P;
}

}  // extern "C"

namespace {

// One pixel's forward compositing over an ordered candidate list
// (Eq. (1) with the readings above).  Records the blended Gaussians so the
// backward can walk them in reverse.  Returns the flag "a decision was within
// the band of its threshold".
struct Blend {
  int idx;       // Gaussian index
  int pos;       // position in the candidate list
  double alpha, T, G, dx, dy;
  bool clamped;
};

// Kinds of a decision taken within the band of its threshold (reported by
// ora_flag_decisions): the 0.99 clamp, the 1/255 skip, the 1e-4 stop.
enum { kDecClamp = 1, kDecSkip = 2, kDecStop = 4 };

int composite_pixel(double sx, double sy, const uint32_t* list, int64_t count,
                    const double* mean2d, const double* conic, const double* opacity,
                    const double* rgb, const double* depth, const double* bg,
                    double out_c[3], double* out_d, double* out_T, int* out_last,
                    std::vector<Blend>* rec,
                    std::vector<std::pair<int, int>>* decisions = nullptr,
                    bool flip_band = false) {
  double T = 1.0, C[3] = {0, 0, 0}, D = 0.0;
  int last = 0, flag = 0;
  // near(): the decision is within the band; with flip_band the other branch
  // is taken (what a computation within rounding of the threshold may do)
  auto near = [&](int i, int kind) {
    flag = 1;
    if (decisions) decisions->push_back({i, kind});
    return flip_band;
  };
  for (int64_t j = 0; j < count; ++j) {
    const int i = (int)list[j];
    const double dx = mean2d[2 * i] - sx, dy = mean2d[2 * i + 1] - sy;
    const double a = conic[3 * i], b = conic[3 * i + 1], c = conic[3 * i + 2];
    const double power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy;
    if (power > 0.0) continue;
    const double G = std::exp(power);
    const double oG = opacity[i] * G;
    bool flip = std::fabs(oG - kAlphaMax) <= kBand * kAlphaMax && near(i, kDecClamp);
    const bool clamped = (oG > kAlphaMax) != flip;
    const double alpha = clamped ? kAlphaMax : oG;
    flip = std::fabs(alpha - kAlphaMin) <= kBand * kAlphaMin && near(i, kDecSkip);
    if ((alpha < kAlphaMin) != flip) continue;
    const double Tn = T * (1.0 - alpha);
    flip = std::fabs(Tn - kTransmittanceMin) <= kBand * kTransmittanceMin && near(i, kDecStop);
    if ((Tn < kTransmittanceMin) != flip) break;
    if (rec) rec->push_back({i, (int)j, alpha, T, G, dx, dy, clamped});
    for (int ch = 0; ch < 3; ++ch) C[ch] += rgb[3 * i + ch] * alpha * T;
    D += depth[i] * alpha * T;
    T = Tn;
    last = (int)j + 1;
  }
  for (int ch = 0; ch < 3; ++ch) out_c[ch] = C[ch] + T * bg[ch];
  *out_d = D;
  *out_T = T;
  *out_last = last;
  return flag;
}

}  // namespace

extern "C" {

// Tiled forward render of one view from a sorted pair list.
// color [3,H,W] planar, depth/T_final [H,W], last [H,W] (position + 1 of the
// last blended Gaussian in the pixel's tile list), flag [H,W].
void ora_render_fwd(int width, int height, int tw, int th,
                    const double* mean2d, const double* conic, const double* opacity,
                    const double* rgb, const double* depth, const uint32_t* vals,
                    const uint32_t* ranges, const double* bg,
                    double* color, double* out_depth, double* T_final, int32_t* last,
                    int32_t* flag, int flip_band) {
  const int tiles_x = (width + tw - 1) / tw;
  const int64_t npx = (int64_t)width * height;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < npx; ++p) {
    const int px = (int)(p % width), py = (int)(p / width);
    const int tile = (py / th) * tiles_x + (px / tw);
    const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
    double c[3], d, T;
    int l;
    flag[p] = composite_pixel(px + 0.5, py + 0.5, vals + s, (int64_t)e - s, mean2d, conic,
                              opacity, rgb, depth, bg, c, &d, &T, &l, nullptr, nullptr,
                              flip_band != 0);
    for (int ch = 0; ch < 3; ++ch) color[ch * npx + p] = c[ch];
    out_depth[p] = d;
    T_final[p] = T;
    last[p] = l;
  }
}

// Decisions within the band of their thresholds, for the parity tests'
// exclusions (no arithmetic beyond the forward's own).  For every pixel with
// at least one such decision: one (pixel, Gaussian, kind) triple per
// decision (kind kDecClamp / kDecSkip / kDecStop), then one (pixel,
// Gaussian, 8) triple per Gaussian blended at that pixel.  Writes at most
// cap triples; returns the number there are.
int64_t ora_flag_decisions(int width, int height, int tw, int th, const double* mean2d,
                           const double* conic, const double* opacity, const double* rgb,
                           const double* depth, const uint32_t* vals, const uint32_t* ranges,
                           const double* bg, int64_t cap, int32_t* out_pix, int32_t* out_gauss,
                           int32_t* out_kind) {
  const int tiles_x = (width + tw - 1) / tw;
  const int64_t npx = (int64_t)width * height;
  int64_t total = 0;
  for (int64_t p = 0; p < npx; ++p) {
    const int px = (int)(p % width), py = (int)(p / width);
    const int tile = (py / th) * tiles_x + (px / tw);
    const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
    double c[3], d, T;
    int l;
    std::vector<Blend> rec;
    std::vector<std::pair<int, int>> dec;
    composite_pixel(px + 0.5, py + 0.5, vals + s, (int64_t)e - s, mean2d, conic, opacity, rgb,
                    depth, bg, c, &d, &T, &l, &rec, &dec);
    if (dec.empty()) continue;
    auto put = [&](int g, int kind) {
      if (total < cap) {
        out_pix[total] = (int32_t)p;
        out_gauss[total] = g;
        out_kind[total] = kind;
      }
      ++total;
    };
    for (const auto& x : dec) put(x.first, x.second);
    for (const Blend& b : rec) put(b.idx, 8);
  }
  return total;
}

// Untiled brute force: every visible Gaussian, ordered by (float32 depth,
// index), for every pixel.  n_blended gets the number of blended Gaussians.
void ora_render_untiled(int width, int height, int64_t n, const int32_t* status,
                        const double* mean2d, const double* conic, const double* opacity,
                        const double* rgb, const double* depth, const float* depth32,
                        const double* bg, double* color, double* out_depth, double* T_final,
                        int32_t* n_blended) {
  std::vector<uint32_t> order;
  for (int64_t i = 0; i < n; ++i)
    if (status[i] == 1) order.push_back((uint32_t)i);
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return depth32[a] < depth32[b]; });
  const int64_t npx = (int64_t)width * height;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t p = 0; p < npx; ++p) {
    const int px = (int)(p % width), py = (int)(p / width);
    std::vector<Blend> rec;
    double c[3], d, T;
    int l;
    composite_pixel(px + 0.5, py + 0.5, order.data(), (int64_t)order.size(), mean2d, conic,
                    opacity, rgb, depth, bg, c, &d, &T, &l, &rec);
    for (int ch = 0; ch < 3; ++ch) color[ch * npx + p] = c[ch];
    out_depth[p] = d;
    T_final[p] = T;
    n_blended[p] = (int32_t)rec.size();
  }
}

// Backward of the tiled render of one view (Eqs. (2)-(4)): per pixel, the
// blended Gaussians are walked back to front; per-pair gradients are summed
// over pixels.  dL_dcolor [3,H,W], dL_ddepth [H,W] (may be null).
// Outputs per Gaussian (FP64, overwritten): g_mean2d [n,2], g_conic [n,3]
// (w.r.t. a, b, c of power = -(a dx^2 + c dy^2)/2 - b dx dy), g_opacity [n],
// g_rgb [n,3], g_depth [n].
void ora_render_bwd(int width, int height, int tw, int th, int64_t n, int64_t n_pairs,
                    const double* mean2d, const double* conic, const double* opacity,
                    const double* rgb, const double* depth, const uint32_t* vals,
                    const uint32_t* ranges, const double* bg, const double* dL_dcolor,
                    const double* dL_ddepth, double* g_mean2d, double* g_conic,
                    double* g_opacity, double* g_rgb, double* g_depth, int flip_band) {
  const int tiles_x = (width + tw - 1) / tw;
  const int tiles_y = (height + th - 1) / th;
  const int64_t npx = (int64_t)width * height;
  // per-pair partial sums (10 values), written by the tile that owns the pair
  std::vector<double> part((size_t)n_pairs * 10, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int tile = 0; tile < tiles_x * tiles_y; ++tile) {
    const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
    const int tx0 = (tile % tiles_x) * tw, ty0 = (tile / tiles_x) * th;
    std::vector<Blend> rec;
    for (int py = ty0; py < std::min(height, ty0 + th); ++py)
      for (int px = tx0; px < std::min(width, tx0 + tw); ++px) {
        const int64_t p = (int64_t)py * width + px;
        rec.clear();
        double c[3], d, Tf;
        int l;
        composite_pixel(px + 0.5, py + 0.5, vals + s, (int64_t)e - s, mean2d, conic, opacity,
                        rgb, depth, bg, c, &d, &Tf, &l, &rec, nullptr, flip_band != 0);
        const double gC[3] = {dL_dcolor[p], dL_dcolor[npx + p], dL_dcolor[2 * npx + p]};
        const double gD = dL_ddepth ? dL_ddepth[p] : 0.0;
        double Sc[3] = {Tf * bg[0], Tf * bg[1], Tf * bg[2]};
        double Sd = 0.0;
        for (int r = (int)rec.size() - 1; r >= 0; --r) {
          const Blend& B = rec[r];
          const int i = B.idx;
          double* g = &part[(size_t)(s + B.pos) * 10];
          const double w = B.alpha * B.T;
          for (int ch = 0; ch < 3; ++ch) g[ch] += w * gC[ch];
          g[3] += w * gD;
          double g_alpha = 0;
          for (int ch = 0; ch < 3; ++ch)
            g_alpha += gC[ch] * (rgb[3 * i + ch] * B.T - Sc[ch] / (1.0 - B.alpha));
          g_alpha += gD * (depth[i] * B.T - Sd / (1.0 - B.alpha));
          for (int ch = 0; ch < 3; ++ch) Sc[ch] += rgb[3 * i + ch] * w;
          Sd += depth[i] * w;
          if (!B.clamped) {
            g[4] += B.G * g_alpha;
            const double g_pow = B.alpha * g_alpha;
            const double a = conic[3 * i], b = conic[3 * i + 1], cc = conic[3 * i + 2];
            g[5] += g_pow * (-0.5 * B.dx * B.dx);
            g[6] += g_pow * (-B.dx * B.dy);
            g[7] += g_pow * (-0.5 * B.dy * B.dy);
            g[8] += g_pow * (-(a * B.dx + b * B.dy));
            g[9] += g_pow * (-(b * B.dx + cc * B.dy));
          }
        }
      }
  }
  for (int64_t i = 0; i < n; ++i) {
    g_mean2d[2 * i] = g_mean2d[2 * i + 1] = 0;
    g_conic[3 * i] = g_conic[3 * i + 1] = g_conic[3 * i + 2] = 0;
    g_rgb[3 * i] = g_rgb[3 * i + 1] = g_rgb[3 * i + 2] = 0;
    g_opacity[i] = 0;
    g_depth[i] = 0;
  }
  for (int64_t j = 0; j < n_pairs; ++j) {
    const uint32_t i = vals[j];
    const double* g = &part[(size_t)j * 10];
    for (int ch = 0; ch < 3; ++ch) g_rgb[3 * i + ch] += g[ch];
    g_depth[i] += g[3];
    g_opacity[i] += g[4];
    for (int k = 0; k < 3; ++k) g_conic[3 * i + k] += g[5 + k];
    g_mean2d[2 * i] += g[8];
    g_mean2d[2 * i + 1] += g[9];
  }
}

// Chain rule from the per-Gaussian 2D gradients of one view to the
// parameters (means, log-scales, quaternions, opacity logits, SH) and to the
// camera tangent xi = (rho, phi).  Parameter gradients are ADDED to the
// outputs (so views can be summed); g_pose[6] is overwritten.
void ora_project_bwd(int64_t n, int deg, const double* means, const double* log_scales,
                     const double* quats, const double* logits, const double* sh,
                     const double* cam20, int width, int height, int tw, int th,
                     int cutoff_3sigma, const double* g_mean2d, const double* g_conic, const double* g_opacity,
                     const double* g_rgb, const double* g_depth, double* g_means,
                     double* g_log_scales, double* g_quats, double* g_logits, double* g_sh,
                     double* g_pose) {
  const Cam cam = load_cam(cam20, width, height);
  const int K = (deg + 1) * (deg + 1);
  std::vector<double> pose_part((size_t)n * 6, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Proj P;
    project_one(i, deg, means, log_scales, quats, logits, sh, cam, tw, th, cutoff_3sigma, P);
    if (P.status != 1) continue;
    const double* W = cam.R;
    // ---- conic (a, b, c) -> Sigma' = X, via dL/dX = -Y G_Y Y, Y = X^-1
    const double ga = g_conic[3 * i], gb = g_conic[3 * i + 1], gc = g_conic[3 * i + 2];
    const double Y[4] = {P.conic[0], P.conic[1], P.conic[1], P.conic[2]};
    const double GY[4] = {ga, 0.5 * gb, 0.5 * gb, gc};
    double tmp[4], GX[4];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) tmp[2 * r + c] = Y[2 * r] * GY[c] + Y[2 * r + 1] * GY[2 + c];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) GX[2 * r + c] = -(tmp[2 * r] * Y[c] + tmp[2 * r + 1] * Y[2 + c]);
    // ---- X = T2 Sigma T2^T + dilation:  G_Sigma = T2^T GX T2, G_T2 = 2 GX T2 Sigma
    double GSigma[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) acc += P.T2[3 * r + a] * GX[2 * r + c] * P.T2[3 * c + b];
        GSigma[3 * a + b] = acc;
      }
    double GT2[6];
    for (int r = 0; r < 2; ++r)
      for (int b = 0; b < 3; ++b) {
        double acc = 0;
        for (int c = 0; c < 2; ++c)
          for (int a = 0; a < 3; ++a) acc += 2.0 * GX[2 * r + c] * P.T2[3 * c + a] * P.Sigma[3 * a + b];
        GT2[3 * r + b] = acc;
      }
    // T2 = J W  ->  G_J = G_T2 W^T
    double GJ[6];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int b = 0; b < 3; ++b) acc += GT2[3 * r + b] * W[3 * k + b];
        GJ[3 * r + k] = acc;
      }
    // ---- camera-space mean t: through J, the 2D mean and the depth
    const double tx = P.tc[0], ty = P.tc[1], tz = P.tc[2];
    double gt[3] = {0, 0, 0};
    gt[2] += GJ[0] * (-cam.fx / (tz * tz)) + GJ[4] * (-cam.fy / (tz * tz));
    if (!P.clamp_u) {  // J02 = -fx tx / tz^2
      gt[0] += GJ[2] * (-cam.fx / (tz * tz));
      gt[2] += GJ[2] * (2.0 * cam.fx * tx / (tz * tz * tz));
    } else {           // J02 = -fx u / tz, u constant
      gt[2] += GJ[2] * (cam.fx * P.u / (tz * tz));
    }
    if (!P.clamp_v) {
      gt[1] += GJ[5] * (-cam.fy / (tz * tz));
      gt[2] += GJ[5] * (2.0 * cam.fy * ty / (tz * tz * tz));
    } else {
      gt[2] += GJ[5] * (cam.fy * P.v / (tz * tz));
    }
    const double gmx = g_mean2d[2 * i], gmy = g_mean2d[2 * i + 1];
    gt[0] += gmx * cam.fx / tz;
    gt[1] += gmy * cam.fy / tz;
    gt[2] += -gmx * cam.fx * tx / (tz * tz) - gmy * cam.fy * ty / (tz * tz);
    gt[2] += g_depth[i];
    // ---- colour: clamp, SH coefficients and the view direction
    double Yb[16], dYb[16][3];
    sh_basis(P.dir[0], P.dir[1], P.dir[2], Yb);
    sh_basis_grad(P.dir[0], P.dir[1], P.dir[2], dYb);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      const double gcr = (P.rgb_raw[ch] < 0) ? 0.0 : g_rgb[3 * i + ch];
      for (int k = 0; k < K; ++k) {
        g_sh[((size_t)i * K + k) * 3 + ch] += Yb[k] * gcr;
        const double coef = sh[((size_t)i * K + k) * 3 + ch];
        for (int r = 0; r < 3; ++r) gdir[r] += gcr * coef * dYb[k][r];
      }
    }
    const double ddot = gdir[0] * P.dir[0] + gdir[1] * P.dir[1] + gdir[2] * P.dir[2];
    double gv[3];
    for (int r = 0; r < 3; ++r) gv[r] = (gdir[r] - ddot * P.dir[r]) / P.dist;
    // ---- means
    for (int r = 0; r < 3; ++r)
      g_means[3 * i + r] += W[r] * gt[0] + W[3 + r] * gt[1] + W[6 + r] * gt[2] + gv[r];
    // ---- covariance Sigma = M M^T, M = R diag(s)
    double M[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[3 * r + c] = P.Rq[3 * r + c] * P.s[c];
    double GM[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += 2.0 * GSigma[3 * r + k] * M[3 * k + c];
        GM[3 * r + c] = acc;
      }
    for (int j = 0; j < 3; ++j) {
      double gs = 0;
      for (int r = 0; r < 3; ++r) gs += GM[3 * r + j] * P.Rq[3 * r + j];
      g_log_scales[3 * i + j] += gs * P.s[j];
    }
    double GR[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) GR[3 * r + c] = GM[3 * r + c] * P.s[c];
    double dR[4][9];
    quat_to_rot_grad(P.q, dR);
    double gqn[4];
    for (int k = 0; k < 4; ++k) {
      double acc = 0;
      for (int e = 0; e < 9; ++e) acc += GR[e] * dR[k][e];
      gqn[k] = acc;
    }
    const double qd = gqn[0] * P.q[0] + gqn[1] * P.q[1] + gqn[2] * P.q[2] + gqn[3] * P.q[3];
    for (int k = 0; k < 4; ++k) g_quats[4 * i + k] += (gqn[k] - qd * P.q[k]) / P.qnorm;
    // ---- opacity logit
    g_logits[i] += g_opacity[i] * P.opacity * (1.0 - P.opacity);
    // ---- camera tangent (left perturbation in the camera frame)
    double* gp = &pose_part[(size_t)i * 6];
    for (int r = 0; r < 3; ++r)
      gp[r] = gt[r] + (W[3 * r] * gv[0] + W[3 * r + 1] * gv[1] + W[3 * r + 2] * gv[2]);
    // t x g_t
    gp[3] = ty * gt[2] - tz * gt[1];
    gp[4] = tz * gt[0] - tx * gt[2];
    gp[5] = tx * gt[1] - ty * gt[0];
    // Sigma_c = W Sigma W^T;  G_Sc = J^T GX J;  g_phi -= 2 axial(Sc G - G Sc)
    double Sc[9], GSc[9], tmp3[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += W[3 * r + k] * P.Sigma[3 * k + c];
        tmp3[3 * r + c] = acc;
      }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += tmp3[3 * r + k] * W[3 * c + k];
        Sc[3 * r + c] = acc;
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double acc = 0;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) acc += P.J[3 * r + a] * GX[2 * r + c] * P.J[3 * c + b];
        GSc[3 * a + b] = acc;
      }
    double A[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double acc = 0;
        for (int k = 0; k < 3; ++k) acc += Sc[3 * r + k] * GSc[3 * k + c] - GSc[3 * r + k] * Sc[3 * k + c];
        A[3 * r + c] = acc;
      }
    gp[3] -= 2.0 * A[7];   // axial(A) = (A21, A02, A10)
    gp[4] -= 2.0 * A[2];
    gp[5] -= 2.0 * A[3];
  }
  for (int k = 0; k < 6; ++k) g_pose[k] = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 6; ++k) g_pose[k] += pose_part[(size_t)i * 6 + k];
}

}  // extern "C"

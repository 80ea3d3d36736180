// a1: per-Gaussian projection for every view (CaRtGS Sec. III-B: primitives
// p, q, s, sigma, SH; alpha comes from a projected 2D Gaussian times the
// opacity).  One thread per Gaussian loops over the views, so the geometry
// parameters are read from HBM once per iteration whatever the batch size;
// SH coefficients are read only when the Gaussian is visible in a view.
// All projection arithmetic is FP64 (the kernel is bound by HBM, and FP64
// runs at the FP32 rate on CDNA vector units).
#include "gs_internal.h"

namespace gs {
namespace {

constexpr double kSH0 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double kSH1 = 0.4886025119029199;    // sqrt(3/(4 pi))
constexpr double kSH2a = 1.0925484305920792;   // sqrt(15/pi)/2
constexpr double kSH2b = 0.31539156525252005;  // sqrt(5/pi)/4
constexpr double kSH2c = 0.5462742152960396;   // sqrt(15/pi)/4
constexpr double kSH3a = 0.5900435899266435;   // sqrt(35/(2 pi))/4
constexpr double kSH3b = 2.890611442640554;    // sqrt(105/pi)/2
constexpr double kSH3c = 0.4570457994644658;   // sqrt(21/(2 pi))/4
constexpr double kSH3d = 0.3731763325901154;   // sqrt(7/pi)/4
constexpr double kSH3e = 1.445305721320277;    // sqrt(105/pi)/4

// Real orthonormal SH with the Condon-Shortley phase at unit direction (x,y,z).
template <int DEG>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double* Y) {
  Y[0] = kSH0;
  if (DEG >= 1) {
    Y[1] = -kSH1 * y;
    Y[2] = kSH1 * z;
    Y[3] = -kSH1 * x;
  }
  if (DEG >= 2) {
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kSH2a * x * y;
    Y[5] = -kSH2a * y * z;
    Y[6] = kSH2b * (2.0 * zz - xx - yy);
    Y[7] = -kSH2a * x * z;
    Y[8] = kSH2c * (xx - yy);
    if (DEG >= 3) {
      Y[9] = -kSH3a * y * (3.0 * xx - yy);
      Y[10] = kSH3b * x * y * z;
      Y[11] = -kSH3c * y * (4.0 * zz - xx - yy);
      Y[12] = kSH3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
      Y[13] = -kSH3c * x * (4.0 * zz - xx - yy);
      Y[14] = kSH3e * z * (xx - yy);
      Y[15] = -kSH3a * x * (xx - 3.0 * yy);
    }
  }
}

__device__ __forceinline__ bool finite_f(float v) { return __builtin_isfinite(v); }


// (three waves per SIMD: at most 168 VGPRs)
template <int DEG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_preprocess(
    const float* __restrict__ means, const float* __restrict__ log_scales,
    const float* __restrict__ quats, const float* __restrict__ logits,
    const float* __restrict__ sh, int64_t n, const float* __restrict__ cams, ViewTable vt,
    uint32_t flags, Rec* __restrict__ rec, ushort4* __restrict__ rect,
    uint32_t* __restrict__ tt, uint32_t* __restrict__ tile_cnt, uint2* __restrict__ chunk_cnt,
    int64_t chunks_per_view, int32_t* __restrict__ fl) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // lanes past the end stay active (as an invalid Gaussian) so that the
  // wavefront reductions at the end see every lane
  const bool in_range = i0 < n;
  const int64_t i = in_range ? i0 : n - 1;

  const float pf[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  const float lf[3] = {log_scales[3 * i], log_scales[3 * i + 1], log_scales[3 * i + 2]};
  const float4 qf = *reinterpret_cast<const float4*>(quats + 4 * i);
  const float bf = logits[i];
  bool ok = finite_f(pf[0]) && finite_f(pf[1]) && finite_f(pf[2]) && finite_f(lf[0]) &&
            finite_f(lf[1]) && finite_f(lf[2]) && finite_f(qf.x) && finite_f(qf.y) &&
            finite_f(qf.z) && finite_f(qf.w) && finite_f(bf);
  int nonfinite = (ok || !in_range) ? 0 : 1;
  ok = ok && in_range;

  // normalised quaternion, rotation, world covariance (symmetric, 6 entries)
  double qw = qf.x, qx = qf.y, qy = qf.z, qz = qf.w;
  const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  ok = ok && (qn > 0.0);
  double S00 = 0, S01 = 0, S02 = 0, S11 = 0, S12 = 0, S22 = 0, o = 0, s2max = 0;
  const double p[3] = {pf[0], pf[1], pf[2]};
  if (ok) {
    // FP64 quotients by a shared denominator as products with its reciprocal
    // (within an ulp of FP64: far below anything the float outputs resolve)
    const double iqn = 1.0 / qn;
    qw *= iqn; qx *= iqn; qy *= iqn; qz *= iqn;
    const double R00 = 1 - 2 * (qy * qy + qz * qz), R01 = 2 * (qx * qy - qw * qz), R02 = 2 * (qx * qz + qw * qy);
    const double R10 = 2 * (qx * qy + qw * qz), R11 = 1 - 2 * (qx * qx + qz * qz), R12 = 2 * (qy * qz - qw * qx);
    const double R20 = 2 * (qx * qz - qw * qy), R21 = 2 * (qy * qz + qw * qx), R22 = 1 - 2 * (qx * qx + qy * qy);
    const double s0 = exp(2.0 * (double)lf[0]), s1 = exp(2.0 * (double)lf[1]), s2 = exp(2.0 * (double)lf[2]);
    S00 = R00 * R00 * s0 + R01 * R01 * s1 + R02 * R02 * s2;
    S01 = R00 * R10 * s0 + R01 * R11 * s1 + R02 * R12 * s2;
    S02 = R00 * R20 * s0 + R01 * R21 * s1 + R02 * R22 * s2;
    S11 = R10 * R10 * s0 + R11 * R11 * s1 + R12 * R12 * s2;
    S12 = R10 * R20 * s0 + R11 * R21 * s1 + R12 * R22 * s2;
    S22 = R20 * R20 * s0 + R21 * R21 * s1 + R22 * R22 * s2;
    o = 1.0 / (1.0 + exp(-(double)bf));
    s2max = fmax(s0, fmax(s1, s2));
  }
  const bool sigma3 = (flags & GS_CUTOFF_3SIGMA) != 0;
  bool sh_loaded = false;
  float shv[K * 3];

  __shared__ uint32_t s_pre[256 / kWave][kWave], s_xy[256 / kWave][kWave], s_w[256 / kWave][kWave];
  for (int v = 0; v < vt.n_views; ++v) {
    const ViewInfo vi = vt.v[v];
    const int64_t ri = (int64_t)v * n + i;
    uint32_t count = 0, box_xy = 0, box_w = 0;
    if (ok) {
      const float* c = cams + (int64_t)v * GS_CAMERA_FLOATS;
      const double fx = c[0], fy = c[1], cx = c[2], cy = c[3];
      const double W0 = c[4], W1 = c[5], W2 = c[6], W3 = c[7], W4 = c[8], W5 = c[9];
      const double W6 = c[10], W7 = c[11], W8 = c[12];
      const double t0 = c[13], t1 = c[14], t2 = c[15], near_z = c[16];
      const double tx = W0 * p[0] + W1 * p[1] + W2 * p[2] + t0;
      const double ty = W3 * p[0] + W4 * p[1] + W5 * p[2] + t1;
      const double tz = W6 * p[0] + W7 * p[1] + W8 * p[2] + t2;
      bool vis = tz > near_z;
      double mx = 0, my = 0, A = 0, B = 0, C = 0, det = 0;
      double j00 = 0, j02 = 0, j11 = 0, j12 = 0;
      if (vis) {
        const double itz = 1.0 / tz;
        mx = fx * tx * itz + cx;
        my = fy * ty * itz + cy;
        const double limx = 1.3 * (double)vi.W / (2.0 * fx);
        const double limy = 1.3 * (double)vi.H / (2.0 * fy);
        const double u = fmin(limx, fmax(-limx, tx * itz));
        const double w = fmin(limy, fmax(-limy, ty * itz));
        // rows of T2 = J W
        j00 = fx * itz; j02 = -fx * u * itz; j11 = fy * itz; j12 = -fy * w * itz;
        if (!sigma3) {
          // Cheap rejection of a Gaussian whose exact tile box cannot reach
          // the image: its half extents are at most kappa_max sqrt(s_max^2
          // |a|^2 + 0.3) (|a|^2 = j00^2 + j02^2 for the orthonormal rows of
          // W, kappa <= sqrt(2 ln 255) < 3.33), taken 1 % and 1 px wider
          // here (plus the float rounding of the mean); the box test below
          // would find the same empty box.
          const float fmx = (float)mx, fmy = (float)my;
          const float hxb = 3.33f * sqrtf((float)(s2max * (j00 * j00 + j02 * j02)) + 0.3f) * 1.01f +
                            1.0f + 1e-5f * fabsf(fmx);
          const float hyb = 3.33f * sqrtf((float)(s2max * (j11 * j11 + j12 * j12)) + 0.3f) * 1.01f +
                            1.0f + 1e-5f * fabsf(fmy);
          const float xmax = (float)(vi.tiles_x * vt.tw), ymax = (float)(vi.tiles_y * vt.th);
          vis = !(fmx + hxb < 0.0f || fmx - hxb > xmax || fmy + hyb < 0.0f || fmy - hyb > ymax);
        }
      }
      if (vis) {
        const double a0 = j00 * W0 + j02 * W6, a1 = j00 * W1 + j02 * W7, a2 = j00 * W2 + j02 * W8;
        const double b0 = j11 * W3 + j12 * W6, b1 = j11 * W4 + j12 * W7, b2 = j11 * W5 + j12 * W8;
        // Sigma a, Sigma b
        const double Sa0 = S00 * a0 + S01 * a1 + S02 * a2;
        const double Sa1 = S01 * a0 + S11 * a1 + S12 * a2;
        const double Sa2 = S02 * a0 + S12 * a1 + S22 * a2;
        const double Sb0 = S00 * b0 + S01 * b1 + S02 * b2;
        const double Sb1 = S01 * b0 + S11 * b1 + S12 * b2;
        const double Sb2 = S02 * b0 + S12 * b1 + S22 * b2;
        A = a0 * Sa0 + a1 * Sa1 + a2 * Sa2 + 0.3;
        B = 0.5 * ((a0 * Sb0 + a1 * Sb1 + a2 * Sb2) + (b0 * Sa0 + b1 * Sa1 + b2 * Sa2));
        C = b0 * Sb0 + b1 * Sb1 + b2 * Sb2 + 0.3;
        det = A * C - B * B;
        vis = (det > 0.0) && (o >= 1.0 / 255.0);
      }
      int x0 = 0, y0 = 0, x1 = 0, y1 = 0;
      if (vis) {
        double hx, hy;
        if (sigma3) {
          const double mid = 0.5 * (A + C);
          const double lmax = mid + sqrt(fmax(0.1, mid * mid - det));
          hx = hy = 3.0 * sqrt(lmax);
        } else {
          const double kappa = sqrt(2.0 * log(255.0 * o));
          hx = kappa * sqrt(A);
          hy = kappa * sqrt(C);
        }
        hx = hx * (1.0 + 1e-4) + 1e-3;
        hy = hy * (1.0 + 1e-4) + 1e-3;
        const double tw = vt.tw, th = vt.th;
        // tile sides are powers of two: the products are the exact quotients
        const double itw = 1.0 / tw, ith = 1.0 / th;
        x0 = (int)fmax(0.0, fmin((double)vi.tiles_x, floor((mx - hx) * itw)));
        y0 = (int)fmax(0.0, fmin((double)vi.tiles_y, floor((my - hy) * ith)));
        x1 = (int)fmax(0.0, fmin((double)vi.tiles_x, floor((mx + hx) * itw) + 1.0));
        y1 = (int)fmax(0.0, fmin((double)vi.tiles_y, floor((my + hy) * ith) + 1.0));
        vis = (x1 > x0) && (y1 > y0);
      }
      if (vis && !sh_loaded) {
        // first view in which the Gaussian is visible: fetch and check SH
        sh_loaded = true;
        const float* shp = sh + (int64_t)i * (K * 3);
        bool shok = true;
#pragma unroll
        for (int k = 0; k < K * 3; ++k) {
          shv[k] = shp[k];
          shok = shok && finite_f(shv[k]);
        }
        if (!shok) {
          ok = false;
          vis = false;
          nonfinite = 1;
        }
      }
      if (vis) {
        // view direction from the camera centre c = -W^T t
        const double cxw = -(W0 * t0 + W3 * t1 + W6 * t2);
        const double cyw = -(W1 * t0 + W4 * t1 + W7 * t2);
        const double czw = -(W2 * t0 + W5 * t1 + W8 * t2);
        const double dx = p[0] - cxw, dy = p[1] - cyw, dz = p[2] - czw;
        const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
        double Y[16];
        sh_basis<DEG>(dx * inv, dy * inv, dz * inv, Y);
        float rgb[3];
        uint32_t clamp_mask = 0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < K; ++k) acc += (double)shv[3 * k + ch] * Y[k];
          rgb[ch] = (float)fmax(0.0, acc + 0.5);
          if (acc + 0.5 < 0.0) clamp_mask |= 1u << ch;
        }
        Rec r;
        r.mx = mx;
        r.my = my;
        // eigen form of the conic Q = Sigma'^-1 (FP32 from the FP64
        // covariance): the covariance's eigenvalues sp >= sm = det / sp; the
        // axis (1, t) nearer to x has Q's eigenvalue 1/sp when A >= C, else
        // 1/sm, the other axis the other one
        const float hc = (float)(0.5 * (A - C)), bf = (float)B;
        const float rc = sqrtf(fmaf(hc, hc, bf * bf));
        const float sp = (float)(0.5 * (A + C)) + rc, df = (float)det;
        const bool xl = hc >= 0.0f;
        const float t = rc > 0.0f ? bf / (xl ? hc + rc : hc - rc) : 0.0f;
        // log2(e)/2 / (1 + t^2) / (sp det): 1/sp = that x det, 1/sm = that x sp^2
        const float g = (float)(0.5 * kLog2e) / (fmaf(t, t, 1.0f) * (sp * df));
        r.t = t;
        r.s1 = xl ? g * df : g * (sp * sp);
        r.s2 = xl ? g * (sp * sp) : g * df;
        r.lo = log2f((float)o);
        r.o = (float)o;
        r.pad[0] = r.pad[1] = 0u;
        r.z = (float)tz;
        r.r = rgb[0];
        r.g = rgb[1];
        r.b = rgb[2];
        r.clamp = clamp_mask;
        rec[ri] = r;
        rect[ri] = make_ushort4((unsigned short)x0, (unsigned short)y0, (unsigned short)x1,
                                (unsigned short)y1);
        count = (uint32_t)((x1 - x0) * (y1 - y0));
        box_xy = (uint32_t)x0 | ((uint32_t)y0 << 16);
        box_w = (uint32_t)(x1 - x0);
      }
    }
    if (in_range) tt[ri] = count;
    // pairs per tile, for the binning: the wavefront's pairs are spread over
    // its lanes (a large Gaussian does not serialise its tiles on one lane).
    // The wavefront's 64 Gaussians are one chunk of the binning's record
    // scan: its pair count (at most 64 x 2^22 tiles of a 16384^2 view in
    // 8x8 tiles, so u32) and its number of visible records.
    {
      const int lane = lane_id(), w = threadIdx.x / kWave;
      uint32_t incl = count;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += y;
      }
      const uint32_t total = __shfl(incl, kWave - 1, kWave);
      const uint32_t n_vis = (uint32_t)__popcll(ballot64(count > 0));
      const int64_t chunk = (int64_t)blockIdx.x * (256 / kWave) + w;
      if (lane == 0 && chunk < chunks_per_view)
        chunk_cnt[(int64_t)v * chunks_per_view + chunk] = make_uint2(total, n_vis);
      // (the radix binning finds the per-tile counts in its sorted lists)
      if (total > 0 && !(flags & GS_RADIX_BIN)) {  // uniform over the wavefront
        s_pre[w][lane] = incl - count;
        s_xy[w][lane] = box_xy;
        s_w[w][lane] = box_w;
        wave_lds_sync();
        for (uint32_t q = (uint32_t)lane; q < total; q += kWave) {
          int lo = 0, hi = kWave - 1;  // owner: the last lane whose prefix is <= q
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[w][mid] <= q) lo = mid; else hi = mid - 1;
          }
          const uint32_t k = q - s_pre[w][lo], bw = s_w[w][lo], xy = s_xy[w][lo];
          const int tx = (int)(xy & 0xFFFFu) + (int)(k % bw), ty = (int)(xy >> 16) + (int)(k / bw);
          atomicAdd(&tile_cnt[vi.tile_off + ty * vi.tiles_x + tx], 1u);
        }
        wave_lds_sync();  // before the next view rewrites the tables
      }
    }
  }
  // non-finite Gaussians are rare: one atomic per wave that has any (the
  // visible-record count is taken by the binning's scan, which also publishes
  // this one)
  const uint64_t nf = ballot64(nonfinite != 0);
  if (lane_id() == 0 && nf) atomicAdd(&fl[F_NF_ACC], (int)__popcll(nf));
}

}  // namespace

hipError_t launch_preprocess(const Plan& P, const gs_gaussians& g, const float* cams,
                             void* ws, hipStream_t s) {
  const int threads = 256;
  const int64_t blocks = (P.n + threads - 1) / threads;
  if (blocks == 0) return hipSuccess;
  Rec* rec = ws_at<Rec>(ws, P.off_rec);
  ushort4* rect = ws_at<ushort4>(ws, P.off_rect);
  uint32_t* tt = ws_at<uint32_t>(ws, P.off_tt);
  uint32_t* tile_cnt = ws_at<uint32_t>(ws, P.off_tile_cnt);
  uint2* chunk_cnt = ws_at<uint2>(ws, P.off_chunk_cnt);
  int32_t* fl = ws_at<int32_t>(ws, P.off_flags);
  const uint32_t flags = P.cfg.flags;
#define GS_PRE(D)                                                                          \
  hipLaunchKernelGGL(k_preprocess<D>, dim3((unsigned)blocks), dim3(threads), 0, s, g.means, \
                     g.log_scales, g.quats, g.opacity_logits, g.sh, P.n, cams, P.vt, flags,  \
                     rec, rect, tt, tile_cnt, chunk_cnt, P.chunks_per_view, fl)
  switch (P.deg) {
    case 0: GS_PRE(0); break;
    case 1: GS_PRE(1); break;
    case 2: GS_PRE(2); break;
    default: GS_PRE(3); break;
  }
#undef GS_PRE
  return hipGetLastError();
}

}  // namespace gs

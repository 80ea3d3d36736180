// Spatial order of a Gaussian pool: a data-layout step, not part of an
// iteration.  Neighbouring Gaussians of a view then sit in the same
// wavefronts of the per-Gaussian kernels (projection, binning counts,
// projection backward), whose per-view branches and tile atomics stop
// diverging over the whole pool.  The mapping loop re-orders the pool
// whenever it re-plans after densification.
//
// Order: the Morton code of each mean in the pool's bounding box (10 bits
// per axis), sorted stably (ties keep the index order), so the permutation
// is deterministic.
#include <cfloat>

#include "gs_internal.h"

namespace gs {
hipError_t launch_radix_sort(uint64_t* keys0, uint64_t* keys1, uint32_t* vals0, uint32_t* vals1,
                             const int32_t* cnt, uint32_t* hist, uint32_t* digit_tot,
                             int64_t nb_cap, int key_bits, bool iota, int* which, hipStream_t s);
hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t s);

namespace {

constexpr int kBoxThreads = 256;
constexpr int kBoxBlocks = 256;
constexpr int kMortonBits = 10;

// Per-block bounding boxes of the means (min x y z, max x y z).
__global__ void __launch_bounds__(kBoxThreads) k_box_part(const float* __restrict__ means,
                                                          int64_t n, float* __restrict__ part) {
  __shared__ float s[6][kBoxThreads];
  float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  for (int64_t i = (int64_t)blockIdx.x * kBoxThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBoxThreads)
    for (int d = 0; d < 3; ++d) {
      const float x = means[3 * i + d];
      if (x == x) {  // a NaN mean takes no part in the box
        lo[d] = fminf(lo[d], x);
        hi[d] = fmaxf(hi[d], x);
      }
    }
  for (int d = 0; d < 3; ++d) {
    s[d][threadIdx.x] = lo[d];
    s[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = kBoxThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = fminf(s[d][threadIdx.x], s[d][threadIdx.x + w]);
        s[3 + d][threadIdx.x] = fmaxf(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  // bit b of v to bit 3b
  uint64_t x = v & 0x3FFu;
  x = (x | (x << 16)) & 0x30000FFull;
  x = (x | (x << 8)) & 0x300F00Full;
  x = (x | (x << 4)) & 0x30C30C3ull;
  x = (x | (x << 2)) & 0x9249249ull;
  return x;
}

// Morton code of every mean in the box of the block partials; values are
// the indices 0..n-1.
__global__ void __launch_bounds__(256) k_morton(const float* __restrict__ means, int64_t n,
                                                const float* __restrict__ part, int n_part,
                                                uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals) {
  __shared__ float box[6];
  if (threadIdx.x < 6) {
    float v = threadIdx.x < 3 ? FLT_MAX : -FLT_MAX;
    for (int b = 0; b < n_part; ++b) {
      const float x = part[b * 6 + threadIdx.x];
      v = threadIdx.x < 3 ? fminf(v, x) : fmaxf(v, x);
    }
    box[threadIdx.x] = v;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  constexpr float kCells = (float)((1 << kMortonBits) - 1);
  uint32_t q[3];
  for (int d = 0; d < 3; ++d) {
    const float ext = box[3 + d] - box[d];
    const float x = means[3 * i + d];
    float t = ext > 0.0f ? (x - box[d]) / ext : 0.0f;
    t = (t == t) ? fminf(1.0f, fmaxf(0.0f, t)) : 1.0f;  // NaN last
    q[d] = (uint32_t)(t * kCells);
  }
  keys[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
  vals[i] = (uint32_t)i;
}

// dst[j] = src[perm[j]] for rows of `width` floats.
__global__ void __launch_bounds__(256) k_gather_rows(const float* __restrict__ src,
                                                     const int32_t* __restrict__ perm,
                                                     int64_t n, int width,
                                                     float* __restrict__ dst) {
  const int64_t total = n * width;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / width, c = e - j * width;
    dst[e] = src[(int64_t)perm[j] * width + c];
  }
}

struct OrderTmp {
  size_t k0, k1, v1, part, hist, dtot, cnt, bytes;
};
OrderTmp order_layout(int64_t n) {
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const int64_t nb = n > kSortTile ? (n + kSortTile - 1) / kSortTile : 1;
  OrderTmp t{};
  t.k0 = 0;
  t.k1 = up(t.k0 + (size_t)n * 8 + 8);
  t.v1 = up(t.k1 + (size_t)n * 8 + 8);
  t.part = up(t.v1 + (size_t)n * 4 + 4);
  t.hist = up(t.part + (size_t)kBoxBlocks * 6 * 4);
  t.dtot = up(t.hist + (size_t)kRadix * nb * 4);
  t.cnt = up(t.dtot + kRadix * 4);
  t.bytes = up(t.cnt + 16);
  return t;
}

}  // namespace

size_t spatial_order_tmp_bytes(int64_t n) { return n < 0 ? 0 : order_layout(n).bytes; }

// perm: [n] int32 output (the Gaussian at new position j is the old perm[j]).
hipError_t launch_spatial_order(const float* means, int64_t n, int32_t* perm, void* tmp,
                                hipStream_t s) {
  const OrderTmp L = order_layout(n);
  char* b = static_cast<char*>(tmp);
  uint64_t* k0 = reinterpret_cast<uint64_t*>(b + L.k0);
  uint64_t* k1 = reinterpret_cast<uint64_t*>(b + L.k1);
  uint32_t* v1 = reinterpret_cast<uint32_t*>(b + L.v1);
  float* part = reinterpret_cast<float*>(b + L.part);
  uint32_t* hist = reinterpret_cast<uint32_t*>(b + L.hist);
  uint32_t* dtot = reinterpret_cast<uint32_t*>(b + L.dtot);
  int32_t* cnt = reinterpret_cast<int32_t*>(b + L.cnt);
  const int nbox = (int)std::min<int64_t>(kBoxBlocks, (n + kBoxThreads - 1) / kBoxThreads);
  hipLaunchKernelGGL(k_box_part, dim3(nbox), dim3(kBoxThreads), 0, s, means, n, part);
  // the permutation doubles as the sort's value buffer
  uint32_t* v0 = reinterpret_cast<uint32_t*>(perm);
  hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, means, n,
                     part, nbox, k0, v0);
  hipError_t e = launch_set_i32(cnt, (int32_t)n, s);
  if (e != hipSuccess) return e;
  const int64_t nb = std::max<int64_t>(1, (n + kSortTile - 1) / kSortTile);
  int which = 0;
  e = launch_radix_sort(k0, k1, v0, v1, cnt, hist, dtot, nb, 3 * kMortonBits, false, &which, s);
  if (e == hipSuccess && which == 1)
    e = hipMemcpyAsync(v0, v1, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_gather_rows(const float* src, const int32_t* perm, int64_t n, int width,
                              float* dst, hipStream_t s) {
  const int64_t total = n * width;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks), dim3(256), 0, s, src, perm, n, width, dst);
  return hipGetLastError();
}

}  // namespace gs

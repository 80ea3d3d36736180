// a2: tile binning.  Pairs are the (Gaussian, tile) incidences of the exact
// tile boxes; their keys are (global tile id << 32 | float32 bits of depth)
// and their values the pair's index in generation order (Gaussian-major,
// row-major tiles).  A stable LSD radix sort (8-bit digits, only the key
// bits in use) therefore orders pairs by (tile, depth, Gaussian): the order
// is unique and the result bit-exact.  Per-tile [start, end) ranges and the
// record index of every sorted pair follow.
//
// Sort structure per digit pass (no spin-waits, no inter-block
// dependencies inside a kernel): upsweep (per-block digit histogram),
// per-digit scan over blocks, downsweep (stable in-block ranking with
// wave64 ballots, scatter).  Pair counts live on the device, so the grid is
// sized for the plan's capacity and blocks past the count exit at once; the
// whole sequence is graph-capturable.
#include "gs_internal.h"

namespace gs {
namespace {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void k_set_i32(int32_t* __restrict__ p, int32_t value) { *p = value; }

// ---------------------------------------------------------------- record scan
// Block-local exclusive scan of tiles_touched; block totals to scan_tmp.
// Sums are 64-bit: a local offset is stored as u32, which is exact whenever
// the total fits the pair capacity (< 2^31); otherwise the overflow flag
// stops every consumer.
__global__ void __launch_bounds__(kScanThreads) k_scan_local(const uint32_t* __restrict__ tt,
                                                             uint32_t* __restrict__ poff,
                                                             uint64_t* __restrict__ block_tot,
                                                             int64_t n) {
  __shared__ uint64_t wsum[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < n ? tt[idx] : 0u;
    s += v[k];
  }
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint64_t incl = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint64_t woff = 0;
  for (int k = 0; k < w; ++k) woff += wsum[k];
  uint64_t run = woff + incl - s;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) poff[idx] = (uint32_t)run;
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) block_tot[blockIdx.x] = run;
}

// Exclusive scan of the block totals (one block), total pair count and the
// capacity check.
__global__ void __launch_bounds__(1024) k_scan_totals(uint64_t* __restrict__ block_tot,
                                                      int64_t nblocks, int64_t cap,
                                                      int32_t* __restrict__ fl) {
  __shared__ uint64_t wsum[1024 / kWave];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (int64_t base = 0; base < nblocks; base += 1024) {
    const int64_t idx = base + threadIdx.x;
    const uint64_t x = idx < nblocks ? block_tot[idx] : 0ull;
    uint64_t incl = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint64_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t woff = carry;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    if (idx < nblocks) block_tot[idx] = woff + incl - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry = woff + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const uint64_t total = carry;
    const bool over = total > (uint64_t)cap;
    fl[F_OVERFLOW] = over ? 1 : 0;
    fl[F_PAIRS] = over ? 0 : (int32_t)total;
    fl[F_PAIRS_WANTED] = total > 0x7FFFFFFFull ? 0x7FFFFFFF : (int32_t)total;
  }
}

// ---------------------------------------------------------------- duplicate
__global__ void __launch_bounds__(256) k_duplicate(
    const uint32_t* __restrict__ tt, uint32_t* __restrict__ poff,
    const uint64_t* __restrict__ block_pre, const ushort4* __restrict__ rect,
    const Rec* __restrict__ rec, int64_t n, int64_t n_rec, ViewTable vt,
    const int32_t* __restrict__ fl, uint64_t* __restrict__ keys,
    uint32_t* __restrict__ pair_rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rec || fl[F_OVERFLOW]) return;
  const uint32_t c = tt[i];
  if (c == 0) return;
  const uint64_t base64 = (uint64_t)poff[i] + block_pre[i / kScanTile];
  if (base64 + c > (uint64_t)fl[F_PAIRS]) return;  // cannot happen without overflow
  const uint32_t base = (uint32_t)base64;
  poff[i] = base;
  const int v = (int)(i / n);
  const ushort4 r = rect[i];
  const uint32_t dbits = __float_as_uint(rec[i].z);
  const int tx = vt.v[v].tiles_x;
  const uint32_t toff = (uint32_t)vt.v[v].tile_off;
  uint32_t o = base;
  for (int y = r.y; y < r.w; ++y)
    for (int x = r.x; x < r.z; ++x) {
      const uint64_t tile = (uint64_t)(toff + (uint32_t)(y * tx + x));
      keys[o] = (tile << 32) | dbits;
      pair_rec[o] = (uint32_t)i;
      ++o;
    }
}

// ---------------------------------------------------------------- radix sort
__device__ __forceinline__ int sort_count(const int32_t* cnt) { return *cnt; }

// Up to this many sort blocks (1M keys) the per-digit scan runs inside the
// downsweep instead of as its own launch.
constexpr int64_t kFusedScanBlocks = 256;

__global__ void __launch_bounds__(kSortThreads) k_radix_upsweep(const uint64_t* __restrict__ keys,
                                                                const int32_t* __restrict__ cnt,
                                                                uint32_t* __restrict__ hist,
                                                                int64_t nb_cap, int shift) {
  const int P = sort_count(cnt);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= P) return;
  __shared__ uint32_t h[kSortThreads / kWave][kRadix];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int k = threadIdx.x; k < (kSortThreads / kWave) * kRadix; k += kSortThreads)
    (&h[0][0])[k] = 0;
  __syncthreads();
#pragma unroll 4
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + (int64_t)w * (kWave * kSortItems) + r * kWave + lane;
    if (idx < P) {
      const uint32_t d = (uint32_t)(keys[idx] >> shift) & (kRadix - 1);
      atomicAdd(&h[w][d], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kSortThreads / kWave; ++k) s += h[k][d];
    hist[(int64_t)d * nb_cap + blockIdx.x] = s;
  }
}

// One block per digit: exclusive scan over the active blocks of that digit.
__global__ void __launch_bounds__(256) k_radix_scan(uint32_t* __restrict__ hist,
                                                    const int32_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ digit_tot,
                                                    int64_t nb_cap) {
  const int P = sort_count(cnt);
  const int64_t nb = (P + kSortTile - 1) / kSortTile;
  uint32_t* row = hist + (int64_t)blockIdx.x * nb_cap;
  __shared__ uint32_t wsum[256 / kWave];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (int64_t base = 0; base < nb; base += 256) {
    const int64_t idx = base + threadIdx.x;
    const uint32_t x = idx < nb ? row[idx] : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t woff = carry;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    if (idx < nb) row[idx] = woff + incl - x;
    __syncthreads();
    if (threadIdx.x == 255) carry = woff + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// Stable in-block ranking and scatter.  Keys of a block are processed in
// rounds of 64 per wave, in index order; lanes holding the same digit in a
// round are found with 8 ballots (one per digit bit); the lowest such lane
// advances the wave's counter for that digit.  Ranks are thus increasing in
// index within each digit: the pass is stable.
// FUSED: the per-digit scan over blocks is done here (each thread sums the
// counts of its digit over the active blocks), for small block counts.
template <bool FUSED>
__global__ void __launch_bounds__(kSortThreads) k_radix_downsweep(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const int32_t* __restrict__ cnt, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ digit_tot, int64_t nb_cap, int shift, int iota_vals) {
  const int P = sort_count(cnt);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= P) return;
  constexpr int NW = kSortThreads / kWave;
  __shared__ uint32_t wcnt[NW][kRadix];
  __shared__ uint32_t boff[kRadix];
  __shared__ uint32_t dsum[NW];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int k = threadIdx.x; k < NW * kRadix; k += kSortThreads) (&wcnt[0][0])[k] = 0;
  // block offset of each digit: exclusive scan of the digit totals plus this
  // block's exclusive prefix within the digit
  {
    const int d = threadIdx.x;  // kSortThreads == kRadix
    uint32_t x, before;
    if (FUSED) {
      const int64_t nb = (P + kSortTile - 1) / kSortTile;
      const uint32_t* row = hist + (int64_t)d * nb_cap;
      uint32_t tot = 0, pre = 0;
      for (int64_t b = 0; b < nb; ++b) {
        const uint32_t h = row[b];
        pre += (b < (int64_t)blockIdx.x) ? h : 0u;
        tot += h;
      }
      x = tot;
      before = pre;
    } else {
      x = digit_tot[d];
      before = hist[(int64_t)d * nb_cap + blockIdx.x];
    }
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) dsum[w] = incl;
    __syncthreads();
    uint32_t woff = 0;
    for (int k = 0; k < w; ++k) woff += dsum[k];
    boff[d] = woff + incl - x + before;
  }
  __syncthreads();

  uint64_t key[kSortItems];
  uint32_t rank[kSortItems];
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + (int64_t)w * (kWave * kSortItems) + r * kWave + lane;
    const bool valid = idx < P;
    key[r] = valid ? keys_in[idx] : 0ull;
    const uint32_t d = (uint32_t)(key[r] >> shift) & (kRadix - 1);
    uint64_t peers = ballot64(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = ballot64(bit);
      peers &= bit ? bb : ~bb;
    }
    uint32_t old = 0;
    if (valid) old = wcnt[w][d];
    const uint64_t below = peers & lt;
    if (valid && below == 0) wcnt[w][d] = old + (uint32_t)__popcll(peers);
    rank[r] = old + (uint32_t)__popcll(below);
  }
  __syncthreads();
  // exclusive prefix over waves, per digit
  {
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const uint32_t c = wcnt[k][d];
      wcnt[k][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t idx = base + (int64_t)w * (kWave * kSortItems) + r * kWave + lane;
    if (idx < P) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & (kRadix - 1);
      const uint32_t pos = boff[d] + wcnt[w][d] + rank[r];
      keys_out[pos] = key[r];
      vals_out[pos] = iota_vals ? (uint32_t)idx : vals_in[idx];
    }
  }
}

// ---------------------------------------------------------------- ranges
__global__ void __launch_bounds__(256) k_ranges(const uint64_t* __restrict__ keys,
                                                const uint32_t* __restrict__ vals,
                                                const uint32_t* __restrict__ pair_rec,
                                                const int32_t* __restrict__ cnt,
                                                uint32_t* __restrict__ ranges,
                                                uint32_t* __restrict__ sorted_rec) {
  const int P = sort_count(cnt);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const uint32_t t = (uint32_t)(keys[i] >> 32);
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[2 * (int64_t)t] = (uint32_t)i;
  if (i == P - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
  sorted_rec[i] = pair_rec[vals[i]];
}

// Work order of the persistent render kernels: tiles by descending pair
// count (16-bit saturated), ties in tile order.
__global__ void __launch_bounds__(256) k_order_keys(const uint32_t* __restrict__ ranges, int T,
                                                    uint64_t* __restrict__ keys,
                                                    int32_t* __restrict__ cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *cnt = T;
  if (t >= T) return;
  const uint32_t c = ranges[2 * (int64_t)t + 1] - ranges[2 * (int64_t)t];
  keys[t] = (uint64_t)(0xFFFFu - (c > 0xFFFFu ? 0xFFFFu : c));
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

// Radix sort of `count` (device int) pairs held in keys[0]/vals[0] over the
// low key_bits bits; ping-pongs through keys[1]/vals[1].  Returns in *which
// the buffer index holding the result.  iota: values are the indices.
hipError_t launch_radix_sort(uint64_t* keys0, uint64_t* keys1, uint32_t* vals0,
                             uint32_t* vals1, const int32_t* cnt, uint32_t* hist,
                             uint32_t* digit_tot, int64_t nb_cap, int key_bits, bool iota,
                             int* which, hipStream_t s) {
  uint64_t* kb[2] = {keys0, keys1};
  uint32_t* vb[2] = {vals0, vals1};
  const int passes = (key_bits + kRadixBits - 1) / kRadixBits;
  int cur = 0;
  const bool fused = nb_cap <= kFusedScanBlocks;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kRadixBits;
    hipLaunchKernelGGL(k_radix_upsweep, dim3((unsigned)nb_cap), dim3(kSortThreads), 0, s,
                       kb[cur], cnt, hist, nb_cap, shift);
    if (fused) {
      hipLaunchKernelGGL(k_radix_downsweep<true>, dim3((unsigned)nb_cap), dim3(kSortThreads), 0, s,
                         kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], cnt, hist, digit_tot, nb_cap,
                         shift, (iota && p == 0) ? 1 : 0);
    } else {
      hipLaunchKernelGGL(k_radix_scan, dim3(kRadix), dim3(256), 0, s, hist, cnt, digit_tot,
                         nb_cap);
      hipLaunchKernelGGL(k_radix_downsweep<false>, dim3((unsigned)nb_cap), dim3(kSortThreads), 0,
                         s, kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], cnt, hist, digit_tot,
                         nb_cap, shift, (iota && p == 0) ? 1 : 0);
    }
    cur ^= 1;
  }
  *which = cur;
  return hipGetLastError();
}

hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const Plan& P, void* ws, hipStream_t s) {
  int32_t* fl = ws_at<int32_t>(ws, P.off_flags);
  uint32_t* tt = ws_at<uint32_t>(ws, P.off_tt);
  uint32_t* poff = ws_at<uint32_t>(ws, P.off_poff);
  uint64_t* btot = ws_at<uint64_t>(ws, P.off_scan);
  uint64_t* keys0 = ws_at<uint64_t>(ws, P.off_keys0);
  uint64_t* keys1 = ws_at<uint64_t>(ws, P.off_keys1);
  uint32_t* vals0 = ws_at<uint32_t>(ws, P.off_vals0);
  uint32_t* vals1 = ws_at<uint32_t>(ws, P.off_vals1);
  uint32_t* pair_rec = ws_at<uint32_t>(ws, P.off_pair_rec);
  uint32_t* sorted_rec = ws_at<uint32_t>(ws, P.off_sorted_rec);
  uint32_t* hist = ws_at<uint32_t>(ws, P.off_hist);
  uint32_t* dtot = ws_at<uint32_t>(ws, P.off_digit_tot);
  uint32_t* ranges = ws_at<uint32_t>(ws, P.off_ranges);
  hipError_t e;
  const int64_t sb = P.scan_blocks;
  if (sb > 0) {
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)sb), dim3(kScanThreads), 0, s, tt, poff,
                       btot, P.n_rec);
  }
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, btot, sb, P.pair_cap, fl);
  if (P.n_rec > 0) {
    const int64_t blocks = (P.n_rec + 255) / 256;
    hipLaunchKernelGGL(k_duplicate, dim3((unsigned)blocks), dim3(256), 0, s, tt, poff, btot,
                       ws_at<ushort4>(ws, P.off_rect), ws_at<Rec>(ws, P.off_rec), P.n, P.n_rec,
                       P.vt, fl, keys0, pair_rec);
  }
  int which = 0;
  e = launch_radix_sort(keys0, keys1, vals0, vals1, fl + F_PAIRS, hist, dtot,
                        P.sort_blocks_cap, P.key_bits, true, &which, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u32(ranges, 0u, 2 * (int64_t)P.vt.total_tiles, s);
  if (e != hipSuccess) return e;
  const uint64_t* ks = which ? keys1 : keys0;
  const uint32_t* vs = which ? vals1 : vals0;
  const int64_t blocks = (P.pair_cap + 255) / 256;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)blocks), dim3(256), 0, s, ks, vs, pair_rec,
                     fl + F_PAIRS, ranges, sorted_rec);
  return hipGetLastError();
}

hipError_t launch_tile_order(const Plan& P, void* ws, hipStream_t s) {
  const int T = P.vt.total_tiles;
  if (T == 0) return hipSuccess;
  char* tmp = ws_at<char>(ws, P.off_order_tmp);
  uint64_t* ka = reinterpret_cast<uint64_t*>(tmp);
  uint64_t* kb = ka + T;
  uint32_t* vb = reinterpret_cast<uint32_t*>(kb + T);
  int32_t* cnt = reinterpret_cast<int32_t*>(vb + T);
  uint32_t* order = ws_at<uint32_t>(ws, P.off_order);
  hipLaunchKernelGGL(k_order_keys, dim3((T + 255) / 256), dim3(256), 0, s,
                     ws_at<uint32_t>(ws, P.off_ranges), T, ka, cnt);
  int which = 0;
  const int64_t nb = (T + kSortTile - 1) / kSortTile;
  // 16 key bits: two passes, the result lands back in (ka, order)
  return launch_radix_sort(ka, kb, order, vb, cnt, ws_at<uint32_t>(ws, P.off_hist),
                           ws_at<uint32_t>(ws, P.off_digit_tot), nb, 16, true, &which, s);
}

// Sorted pair values (original pair indices) after launch_bin_sort.
uint32_t* sorted_vals(const Plan& P, void* ws) {
  const int passes = (P.key_bits + kRadixBits - 1) / kRadixBits;
  return ws_at<uint32_t>(ws, (passes & 1) ? P.off_vals1 : P.off_vals0);
}
uint64_t* sorted_keys(const Plan& P, void* ws) {
  const int passes = (P.key_bits + kRadixBits - 1) / kRadixBits;
  return ws_at<uint64_t>(ws, (passes & 1) ? P.off_keys1 : P.off_keys0);
}

}  // namespace gs

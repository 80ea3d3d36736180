// a2: tile binning.  Pairs are the (Gaussian, tile) incidences of the exact
// tile boxes, numbered in generation order (record-major, row-major tiles
// within a box).  The order the renderer needs is (tile, depth, generation
// index): unique, so the result is bit-exact whatever the schedule.
//
// The projection counts pairs per tile as it computes the boxes.  Then:
// exclusive scans of the per-record pair counts (generation offsets) and of
// the per-tile counts (tile list starts), one scatter that puts every pair
// into its tile's list at an atomically taken slot with the key
// (depth bits << 32 | generation index), and a per-tile sort of those keys
// (one wavefront per tile: a bitonic network in LDS for lists up to 2048,
// an LSD radix sort through global memory beyond).  Five launches whatever
// the pair count, no spin-waits; graph-capturable.
//
// The general stable LSD radix sort (8-bit digits, wave64 ballot ranking)
// below serves the standalone key/value sort and the longest-first tile
// order of the persistent render kernels.
#include "gs_internal.h"

namespace gs {
namespace {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void k_set_i32(int32_t* __restrict__ p, int32_t value) { *p = value; }

__global__ void k_fill2_u32(uint32_t* __restrict__ a, int64_t na, uint32_t* __restrict__ b,
                            int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) a[i] = 0u;
  if (i < nb) b[i] = 0u;
}

// ---------------------------------------------------------------- scans
// Block-local exclusive scan of u32 counts; block totals to block_tot.
// Sums are 64-bit: a local offset is stored as u32, which is exact whenever
// the total fits the pair capacity (< 2^31); otherwise the overflow flag
// stops every consumer.  ZERO: the counts are cleared after reading (the
// tile counters become the scatter's cursors).
template <bool ZERO>
__global__ void __launch_bounds__(kScanThreads) k_scan_local(uint32_t* __restrict__ cnt,
                                                             uint32_t* __restrict__ off,
                                                             uint64_t* __restrict__ block_tot,
                                                             int64_t n) {
  __shared__ uint64_t wsum[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < n ? cnt[idx] : 0u;
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
    if (idx < n) {
      off[idx] = (uint32_t)run;
      if (ZERO) cnt[idx] = 0u;
    }
    run += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) block_tot[blockIdx.x] = run;
}

// In-place exclusive scan of n u64 values by one 1024-thread block; returns
// the total in every thread.
__device__ uint64_t block_scan_u64(uint64_t* __restrict__ a, int64_t n, uint64_t* wsum,
                                   uint64_t* carry) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) *carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t idx = base + threadIdx.x;
    const uint64_t x = idx < n ? a[idx] : 0ull;
    uint64_t incl = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint64_t y = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint64_t woff = *carry;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    if (idx < n) a[idx] = woff + incl - x;
    __syncthreads();
    if (threadIdx.x == 1023) *carry = woff + incl;
    __syncthreads();
  }
  return *carry;
}

// Exclusive scans of the record and tile block totals (one block); total
// pair count and the capacity check.  Both scans count the same pairs; a
// mismatch is reported as an overflow so that nothing is scattered.
__global__ void __launch_bounds__(1024) k_scan_totals(uint64_t* __restrict__ rec_tot,
                                                      int64_t n_rec_blocks,
                                                      uint64_t* __restrict__ tile_tot,
                                                      int64_t n_tile_blocks, int64_t cap,
                                                      int32_t* __restrict__ fl) {
  __shared__ uint64_t wsum[1024 / kWave];
  __shared__ uint64_t carry;
  const uint64_t total = block_scan_u64(rec_tot, n_rec_blocks, wsum, &carry);
  const uint64_t total_t = block_scan_u64(tile_tot, n_tile_blocks, wsum, &carry);
  if (threadIdx.x == 0) {
    const bool over = total > (uint64_t)cap || total != total_t;
    fl[F_OVERFLOW] = over ? 1 : 0;
    fl[F_PAIRS] = over ? 0 : (int32_t)total;
    fl[F_PAIRS_WANTED] = total > 0x7FFFFFFFull ? 0x7FFFFFFF : (int32_t)total;
  }
}

// ---------------------------------------------------------------- scatter
// Thread per record: generation offsets become absolute (poff), every pair
// gets the next free slot of its tile's list with key (depth bits << 32 |
// generation index), and pair -> record is recorded.
__global__ void __launch_bounds__(256) k_scatter(
    const uint32_t* __restrict__ tt, uint32_t* __restrict__ poff,
    const uint64_t* __restrict__ rec_pre, const ushort4* __restrict__ rect,
    const Rec* __restrict__ rec, int64_t n, int64_t n_rec, ViewTable vt,
    const int32_t* __restrict__ fl, const uint32_t* __restrict__ tstart,
    const uint64_t* __restrict__ tile_pre, uint32_t* __restrict__ cursor,
    uint64_t* __restrict__ skey, uint32_t* __restrict__ pair_rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rec || fl[F_OVERFLOW]) return;
  const uint32_t c = tt[i];
  if (c == 0) return;
  const uint64_t P = (uint64_t)fl[F_PAIRS];
  const uint64_t base64 = (uint64_t)poff[i] + rec_pre[i / kScanTile];
  if (base64 + c > P) return;  // cannot happen without overflow
  uint32_t p = (uint32_t)base64;
  poff[i] = p;
  const int v = (int)(i / n);
  const ushort4 r = rect[i];
  const uint64_t dbits = (uint64_t)__float_as_uint(rec[i].z) << 32;
  const int tx = vt.v[v].tiles_x;
  const int toff = vt.v[v].tile_off;
  for (int y = r.y; y < r.w; ++y)
    for (int x = r.x; x < r.z; ++x) {
      const int t = toff + y * tx + x;
      const uint64_t slot = (uint64_t)tstart[t] + tile_pre[t / kScanTile] + atomicAdd(&cursor[t], 1u);
      if (slot < P) skey[slot] = dbits | p;
      pair_rec[p] = (uint32_t)i;
      ++p;
    }
}

// ---------------------------------------------------------------- tile sort
// One wavefront per tile.  Output: sorted keys (tile << 32 | depth bits),
// generation indices, record ids, and the tile's [start, end) range ((0, 0)
// when empty).  Lists up to kTileSortLds keys: bitonic network in LDS.
// Longer lists: LSD radix sort with 8-bit digits over the generation-index
// bits in use and the 32 depth bits, ping-ponging between the scatter
// buffer and the output buffer; each round of 64 keys is ranked with 8
// ballots, so every pass is stable.
__device__ void wave_radix_pass(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                uint32_t n, int shift, uint32_t* hist) {
  const int lane = threadIdx.x;
  for (int d = lane; d < kRadix; d += kWave) hist[d] = 0u;
  __syncthreads();
  for (uint32_t k = lane; k < n; k += kWave)
    atomicAdd(&hist[(uint32_t)(src[k] >> shift) & (kRadix - 1)], 1u);
  __syncthreads();
  // exclusive scan of the 256 bins: 4 per lane
  uint32_t h[kRadix / kWave], sum = 0;
#pragma unroll
  for (int q = 0; q < kRadix / kWave; ++q) {
    h[q] = hist[lane * (kRadix / kWave) + q];
    sum += h[q];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  uint32_t run = incl - sum;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kRadix / kWave; ++q) {
    hist[lane * (kRadix / kWave) + q] = run;
    run += h[q];
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  for (uint32_t b = 0; b < n; b += kWave) {
    const uint32_t k = b + (uint32_t)lane;
    const bool valid = k < n;
    const uint64_t key = valid ? src[k] : 0ull;
    const uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
    uint64_t peers = ballot64(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      const bool on = (d >> bit) & 1u;
      const uint64_t bb = ballot64(on);
      peers &= on ? bb : ~bb;
    }
    uint32_t at = 0;
    if (valid) at = hist[d];
    const uint64_t below = peers & lt;
    if (valid) dst[at + (uint32_t)__popcll(below)] = key;
    __syncthreads();
    if (valid && below == 0) hist[d] = at + (uint32_t)__popcll(peers);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kWave) k_tile_sort(
    const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ tstart,
    const uint64_t* __restrict__ tile_pre, int T, const int32_t* __restrict__ fl,
    uint64_t* __restrict__ skey, const uint32_t* __restrict__ pair_rec,
    uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    uint32_t* __restrict__ sorted_rec, uint32_t* __restrict__ ranges) {
  __shared__ uint64_t sk[kTileSortLds];
  const int t = blockIdx.x;
  const int lane = threadIdx.x;
  const uint64_t P = (uint64_t)fl[F_PAIRS];
  const uint32_t n = fl[F_OVERFLOW] ? 0u : cnt[t];
  const uint64_t start64 = (uint64_t)tstart[t] + tile_pre[t / kScanTile];
  const bool ok = n > 0 && start64 + n <= P;
  if (lane == 0) {
    ranges[2 * (int64_t)t] = ok ? (uint32_t)start64 : 0u;
    ranges[2 * (int64_t)t + 1] = ok ? (uint32_t)(start64 + n) : 0u;
  }
  if (!ok) return;
  const uint32_t start = (uint32_t)start64;
  const uint64_t tkey = (uint64_t)(uint32_t)t << 32;
  if (n <= (uint32_t)kTileSortLds) {
    uint32_t m = kWave;
    while (m < n) m <<= 1;
    for (uint32_t k = lane; k < m; k += kWave) sk[k] = k < n ? skey[start + k] : ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= m; size <<= 1) {
      for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
        for (uint32_t idx = lane; idx < m / 2; idx += kWave) {
          const uint32_t a = 2 * idx - (idx & (stride - 1));
          const uint32_t b = a + stride;
          const uint64_t ka = sk[a], kb = sk[b];
          const bool up = (a & size) == 0;
          if ((ka > kb) == up) {
            sk[a] = kb;
            sk[b] = ka;
          }
        }
        __syncthreads();
      }
    }
    for (uint32_t k = lane; k < n; k += kWave) {
      const uint64_t key = sk[k];
      const uint32_t g = (uint32_t)key;
      keys_out[start + k] = tkey | (key >> 32);
      vals_out[start + k] = g;
      sorted_rec[start + k] = pair_rec[g];
    }
    return;
  }
  // long list: generation-index bits in use, then the 32 depth bits
  uint32_t* hist = reinterpret_cast<uint32_t*>(sk);
  const uint32_t pmax = (uint32_t)(P - 1);
  const int gbits = pmax == 0 ? 1 : 32 - __clz((int)pmax);
  const int gpasses = (gbits + kRadixBits - 1) / kRadixBits;
  uint64_t* a = skey + start;
  uint64_t* b = keys_out + start;
  for (int q = 0; q < gpasses; ++q) {
    wave_radix_pass(a, b, n, q * kRadixBits, hist);
    uint64_t* tmp = a; a = b; b = tmp;
  }
  for (int q = 0; q < 32 / kRadixBits; ++q) {
    wave_radix_pass(a, b, n, 32 + q * kRadixBits, hist);
    uint64_t* tmp = a; a = b; b = tmp;
  }
  // the result is in `a`; the output is written element by element in place
  for (uint32_t k = lane; k < n; k += kWave) {
    const uint64_t key = a[k];
    const uint32_t g = (uint32_t)key;
    keys_out[start + k] = tkey | (key >> 32);
    vals_out[start + k] = g;
    sorted_rec[start + k] = pair_rec[g];
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

hipError_t launch_clear_counters(const Plan& P, void* ws, hipStream_t s) {
  // per-iteration flags 0..3 and the per-tile pair counters
  const int64_t T = P.vt.total_tiles;
  const int64_t m = T > 4 ? T : 4;
  hipLaunchKernelGGL(k_fill2_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                     ws_at<uint32_t>(ws, P.off_flags), (int64_t)4,
                     ws_at<uint32_t>(ws, P.off_tile_cnt), T);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const Plan& P, void* ws, hipStream_t s) {
  int32_t* fl = ws_at<int32_t>(ws, P.off_flags);
  uint32_t* tt = ws_at<uint32_t>(ws, P.off_tt);
  uint32_t* poff = ws_at<uint32_t>(ws, P.off_poff);
  uint64_t* rec_tot = ws_at<uint64_t>(ws, P.off_scan);
  uint32_t* tcnt = ws_at<uint32_t>(ws, P.off_tile_cnt);
  uint32_t* tstart = ws_at<uint32_t>(ws, P.off_tile_start);
  uint64_t* tile_tot = ws_at<uint64_t>(ws, P.off_tile_scan);
  const int T = P.vt.total_tiles;
  const int64_t sb = P.scan_blocks, tb = P.tile_scan_blocks;
  if (sb > 0)
    hipLaunchKernelGGL(k_scan_local<false>, dim3((unsigned)sb), dim3(kScanThreads), 0, s, tt,
                       poff, rec_tot, P.n_rec);
  if (tb > 0)
    hipLaunchKernelGGL(k_scan_local<true>, dim3((unsigned)tb), dim3(kScanThreads), 0, s, tcnt,
                       tstart, tile_tot, (int64_t)T);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, rec_tot, sb, tile_tot, tb,
                     P.pair_cap, fl);
  uint64_t* skey = ws_at<uint64_t>(ws, P.off_scatter);
  uint32_t* pair_rec = ws_at<uint32_t>(ws, P.off_pair_rec);
  if (P.n_rec > 0) {
    const int64_t blocks = (P.n_rec + 255) / 256;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, tt, poff, rec_tot,
                       ws_at<ushort4>(ws, P.off_rect), ws_at<Rec>(ws, P.off_rec), P.n, P.n_rec,
                       P.vt, fl, tstart, tile_tot, tcnt, skey, pair_rec);
  }
  if (T > 0)
    hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)T), dim3(kWave), 0, s, tcnt, tstart, tile_tot,
                       T, fl, skey, pair_rec, ws_at<uint64_t>(ws, P.off_keys),
                       ws_at<uint32_t>(ws, P.off_vals), ws_at<uint32_t>(ws, P.off_sorted_rec),
                       ws_at<uint32_t>(ws, P.off_ranges));
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

// Sorted pair values (generation indices) after launch_bin_sort.
uint32_t* sorted_vals(const Plan& P, void* ws) { return ws_at<uint32_t>(ws, P.off_vals); }

}  // namespace gs

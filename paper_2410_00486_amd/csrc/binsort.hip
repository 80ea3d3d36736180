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
// Block-level exclusive scans of per-element counts (kScanThreads threads x
// kScanItems consecutive elements).  Sums are 64-bit: a block-local offset
// is stored as u32, which is exact whenever the total fits the pair
// capacity (< 2^31); otherwise the overflow flag stops every consumer.

// Exclusive start of this thread's items within the block for a thread sum
// s; the block total goes to *total.  Every thread of the block must call.
__device__ __forceinline__ uint64_t scan_start(uint64_t s, uint64_t* wsum, uint64_t* total) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint64_t incl = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint64_t woff = 0, tot = 0;
  for (int k = 0; k < kScanThreads / kWave; ++k) {
    woff += k < w ? wsum[k] : 0ull;
    tot += wsum[k];
  }
  __syncthreads();  // wsum is reused by the next channel
  *total = tot;
  return woff + incl - s;
}

// Records: pair counts -> generation offsets (poff); visible (non-zero)
// records -> position in the compact visible list (vpre).
__device__ void scan_records(int64_t blk, const uint32_t* __restrict__ tt,
                             uint32_t* __restrict__ poff, uint64_t* __restrict__ rec_tot,
                             uint32_t* __restrict__ vpre, uint64_t* __restrict__ vis_tot,
                             int64_t n, uint64_t* wsum) {
  const int64_t base = blk * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint64_t sp = 0, sv = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < n ? tt[idx] : 0u;
    sp += v[k];
    sv += v[k] > 0 ? 1u : 0u;
  }
  uint64_t tp, tv;
  uint64_t rp = scan_start(sp, wsum, &tp);
  uint64_t rv = scan_start(sv, wsum, &tv);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) {
      poff[idx] = (uint32_t)rp;
      vpre[idx] = (uint32_t)rv;
    }
    rp += v[k];
    rv += v[k] > 0 ? 1u : 0u;
  }
  if (threadIdx.x == 0) {
    rec_tot[blk] = tp;
    vis_tot[blk] = tv;
  }
}

// Tiles: pair counts -> list starts (the counters are cleared and become
// the scatter's cursors).  With the splat-wise backward also the starts of
// each tile's buckets of 64 positions, and its positions in the two bucket
// queues: buckets with more than 32 pairs (all but possibly the last) and
// buckets with at most 32 (possibly the last).
__device__ __forceinline__ void bucket_split(uint32_t c, uint32_t& nb, uint32_t& full,
                                             uint32_t& half) {
  nb = (c + kBucket - 1) / kBucket;
  const uint32_t r = c - (nb > 0 ? (nb - 1) * kBucket : 0u);  // pairs of the last bucket
  half = (c > 0 && r <= 32) ? 1u : 0u;
  full = nb - half;
}

struct TileScanArgs {
  uint32_t* cnt;
  uint32_t* tstart;
  uint64_t* tile_tot;
  int64_t n;
  uint32_t* bstart;
  uint64_t* bucket_tot;
  uint32_t* fstart;
  uint64_t* full_tot;
  uint32_t* hstart;
  uint64_t* half_tot;
};

__device__ void scan_tiles(int64_t blk, const TileScanArgs& A, uint64_t* wsum) {
  uint32_t* __restrict__ cnt = A.cnt;
  uint32_t* __restrict__ tstart = A.tstart;
  uint32_t* __restrict__ bstart = A.bstart;
  uint32_t* __restrict__ fstart = A.fstart;
  uint32_t* __restrict__ hstart = A.hstart;
  const int64_t n = A.n;
  const int64_t base = blk * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint64_t sp = 0, sb = 0, sf = 0, sh = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < n ? cnt[idx] : 0u;
    uint32_t nb, f, h;
    bucket_split(v[k], nb, f, h);
    sp += v[k];
    sb += nb;
    sf += f;
    sh += h;
  }
  uint64_t tp, tb, tf, th;
  uint64_t rp = scan_start(sp, wsum, &tp);
  uint64_t rb = 0, rf = 0, rh = 0;
  if (bstart) {  // uniform
    rb = scan_start(sb, wsum, &tb);
    rf = scan_start(sf, wsum, &tf);
    rh = scan_start(sh, wsum, &th);
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    uint32_t nb, f, h;
    bucket_split(v[k], nb, f, h);
    if (idx < n) {
      tstart[idx] = (uint32_t)rp;
      cnt[idx] = 0u;
      if (bstart) {
        bstart[idx] = (uint32_t)rb;
        fstart[idx] = (uint32_t)rf;
        hstart[idx] = (uint32_t)rh;
      }
    }
    rp += v[k];
    rb += nb;
    rf += f;
    rh += h;
  }
  if (threadIdx.x == 0) {
    A.tile_tot[blk] = tp;
    if (bstart) {
      A.bucket_tot[blk] = tb;
      A.full_tot[blk] = tf;
      A.half_tot[blk] = th;
    }
  }
}

// Block-total arrays of the scans (records: pairs, visible; tiles: pairs,
// buckets, full and half buckets), scanned together by one block.
constexpr int kMaxChannels = 6;
struct ScanChannels {
  uint64_t* a[kMaxChannels];
  int64_t n[kMaxChannels];
  int count;
};

// In-place exclusive scans of up to six u64 arrays at once by one block of
// NT threads (each array has its own length); totals to tot[].
template <int NT>
__device__ void block_scan_channels(const ScanChannels& ch, uint64_t* tot) {
  __shared__ uint64_t wsum[kMaxChannels][NT / kWave];
  __shared__ uint64_t carry[kMaxChannels];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  if (threadIdx.x < kMaxChannels) carry[threadIdx.x] = 0;
  int64_t nmax = 0;
  for (int c = 0; c < ch.count; ++c) nmax = ch.n[c] > nmax ? ch.n[c] : nmax;
  __syncthreads();
  for (int64_t base = 0; base < nmax; base += NT) {
    const int64_t idx = base + threadIdx.x;
    uint64_t x[kMaxChannels], incl[kMaxChannels];
#pragma unroll
    for (int c = 0; c < kMaxChannels; ++c) {
      x[c] = (c < ch.count && idx < ch.n[c]) ? ch.a[c][idx] : 0ull;
      incl[c] = x[c];
    }
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
      for (int c = 0; c < kMaxChannels; ++c) {
        const uint64_t y = __shfl_up(incl[c], o, kWave);
        if (lane >= o) incl[c] += y;
      }
    }
    if (lane == kWave - 1)
      for (int c = 0; c < kMaxChannels; ++c) wsum[c][w] = incl[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kMaxChannels; ++c) {
      uint64_t woff = carry[c];
      for (int k = 0; k < w; ++k) woff += wsum[c][k];
      if (c < ch.count && idx < ch.n[c]) ch.a[c][idx] = woff + incl[c] - x[c];
      if (threadIdx.x == NT - 1) incl[c] = woff + incl[c];  // running total
    }
    __syncthreads();
    if (threadIdx.x == NT - 1)
      for (int c = 0; c < kMaxChannels; ++c) carry[c] = incl[c];
    __syncthreads();
  }
  for (int c = 0; c < kMaxChannels; ++c) tot[c] = carry[c];
}

// From the scanned totals: pair count, capacity check, visible count and
// the sizes of the bucket queues.  Both pair totals count the same pairs; a
// mismatch is reported as an overflow so that nothing is scattered.
__device__ void set_scan_flags(const ScanChannels& ch, const uint64_t* tot, int64_t cap,
                               int32_t* fl) {
  const uint64_t total = tot[0], visible = tot[1], total_t = tot[2];
  const uint64_t n_full = ch.count > 4 ? tot[4] : 0, n_half = ch.count > 5 ? tot[5] : 0;
  const bool over = total > (uint64_t)cap || total != total_t;
  fl[F_OVERFLOW] = over ? 1 : 0;
  fl[F_PAIRS] = over ? 0 : (int32_t)total;
  fl[F_PAIRS_WANTED] = total > 0x7FFFFFFFull ? 0x7FFFFFFF : (int32_t)total;
  fl[F_VISIBLE] = (int32_t)visible;
  // long lists are queued by the tile sort that follows; the bucket queues
  // are filled there at the positions scanned here
  fl[F_LONG_TILES] = 0;
  fl[F_BQ_FULL] = over ? 0 : (int32_t)n_full;
  fl[F_BQ_HALF] = over ? 0 : (int32_t)n_half;
}

// Record blocks first, then tile blocks: one launch for both scans.
// The last block to finish (counted in a flag; each block publishes its
// totals before it counts itself) scans the block totals of all channels.
__global__ void __launch_bounds__(kScanThreads) k_scans(
    const uint32_t* __restrict__ tt, uint32_t* __restrict__ poff, uint64_t* __restrict__ rec_tot,
    uint32_t* __restrict__ vpre, uint64_t* __restrict__ vis_tot, int64_t n_rec,
    int64_t rec_blocks, TileScanArgs tiles, ScanChannels ch, int64_t cap,
    int32_t* __restrict__ fl) {
  __shared__ uint64_t wsum[kScanThreads / kWave];
  __shared__ int is_last;
  if ((int64_t)blockIdx.x < rec_blocks)
    scan_records(blockIdx.x, tt, poff, rec_tot, vpre, vis_tot, n_rec, wsum);
  else
    scan_tiles((int64_t)blockIdx.x - rec_blocks, tiles, wsum);
  if (threadIdx.x == 0) {
    __threadfence();  // this block's totals before its count
    is_last = atomicAdd(&fl[F_SCAN_DONE], 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;  // uniform over the block
  __threadfence();
  uint64_t tot[kMaxChannels];
  block_scan_channels<kScanThreads>(ch, tot);
  if (threadIdx.x == 0) {
    set_scan_flags(ch, tot, cap, fl);
    fl[F_SCAN_DONE] = 0;  // ready for the next binning
  }
}


// ---------------------------------------------------------------- scatter
// Generation offsets become absolute (poff), every pair gets the next free
// slot of its tile's list with key (depth bits << 32 | generation index),
// and pair -> record is recorded.  Each wavefront takes 64 consecutive
// records and spreads their pairs evenly over its lanes (exclusive scan of
// the pair counts, binary search of a pair's record in LDS), so a large
// Gaussian does not serialise its tiles' slot claims on one lane.
__global__ void __launch_bounds__(256) k_scatter(
    const uint32_t* __restrict__ tt, uint32_t* __restrict__ poff,
    const uint64_t* __restrict__ rec_pre, const ushort4* __restrict__ rect,
    const Rec* __restrict__ rec, int64_t n, int64_t n_rec, ViewTable vt,
    const int32_t* __restrict__ fl, const uint32_t* __restrict__ tstart,
    const uint64_t* __restrict__ tile_pre, uint32_t* __restrict__ cursor,
    uint64_t* __restrict__ skey, uint32_t* __restrict__ pair_rec,
    const uint32_t* __restrict__ vpre, const uint64_t* __restrict__ vis_pre,
    uint32_t* __restrict__ vis_list) {
  constexpr int NW = 256 / kWave;
  __shared__ uint32_t s_pre[NW][kWave + 1];
  __shared__ uint32_t s_p0[NW][kWave], s_dbits[NW][kWave], s_x0y0[NW][kWave];
  __shared__ uint32_t s_wv[NW][kWave];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t P = (uint64_t)fl[F_PAIRS];
  const bool over = fl[F_OVERFLOW] != 0;
  uint32_t c = (i < n_rec && !over) ? tt[i] : 0u;
  uint32_t p0 = 0, dbits = 0, x0y0 = 0, wv = 0;
  if (c > 0) {
    const uint64_t base64 = (uint64_t)poff[i] + rec_pre[i / kScanTile];
    if (base64 + c > P) {
      c = 0;  // cannot happen without overflow
    } else {
      p0 = (uint32_t)base64;
      poff[i] = p0;
      vis_list[vpre[i] + vis_pre[i / kScanTile]] = (uint32_t)i;  // records in index order
      const ushort4 r = rect[i];
      dbits = __float_as_uint(rec[i].z);
      x0y0 = (uint32_t)r.x | ((uint32_t)r.y << 16);
      wv = (uint32_t)(r.z - r.x) | ((uint32_t)(i / n) << 16);
    }
  }
  uint32_t incl = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  s_pre[w][lane] = incl - c;
  if (lane == kWave - 1) s_pre[w][kWave] = incl;
  s_p0[w][lane] = p0;
  s_dbits[w][lane] = dbits;
  s_x0y0[w][lane] = x0y0;
  s_wv[w][lane] = wv;
  __syncthreads();
  const uint32_t total = s_pre[w][kWave];
  const int64_t rec0 = (int64_t)blockIdx.x * 256 + (int64_t)w * kWave;
  for (uint32_t q = (uint32_t)lane; q < total; q += kWave) {
    // owner: the last record whose prefix is <= q (it has pairs)
    int lo = 0, hi = kWave - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[w][mid] <= q) lo = mid; else hi = mid - 1;
    }
    const uint32_t k = q - s_pre[w][lo];
    const uint32_t wvj = s_wv[w][lo], xy = s_x0y0[w][lo];
    const uint32_t bw = wvj & 0xFFFFu;
    const int v = (int)(wvj >> 16);
    const int x = (int)(xy & 0xFFFFu) + (int)(k % bw);
    const int y = (int)(xy >> 16) + (int)(k / bw);
    const int t = vt.v[v].tile_off + y * vt.v[v].tiles_x + x;
    const uint32_t p = s_p0[w][lo] + k;
    const uint64_t slot = (uint64_t)tstart[t] + tile_pre[t / kScanTile] + atomicAdd(&cursor[t], 1u);
    if (slot < P) skey[slot] = ((uint64_t)s_dbits[w][lo] << 32) | p;
    pair_rec[p] = (uint32_t)(rec0 + lo);
  }
}

// ---------------------------------------------------------------- tile sort
// Output per tile: sorted keys (tile << 32 | depth bits), generation
// indices, record ids, the [start, end) range ((0, 0) when empty) and, for
// the splat-wise backward, the absolute bucket offset.  Keys are unique, so
// any correct sort gives the same lists.  k_tile_sort (one wavefront per
// tile) sorts lists up to 64 keys in registers (rank = number of smaller
// keys) and up to kTileSortSmall keys with a bitonic network in LDS, and
// queues longer lists; k_tile_sort_long (1024-thread blocks, grid-stride
// over the queue) sorts them with the same network in LDS up to
// kTileSortLong keys and in place in global memory beyond.
//
// The network keeps every merge ascending (the first compare of a merge
// pairs i with its mirror in the block), so positions past the list end
// act as +infinity and are never touched: no padding is written.
constexpr uint32_t kTileSortSmall = 512;
constexpr uint32_t kTileSortLong = 16384;
constexpr int kLongThreads = 1024;

struct TileSortOut {
  uint64_t* keys;
  uint32_t* vals;
  uint32_t* sorted_rec;
  const uint32_t* pair_rec;
  const Rec* rec;
  Rec* lrec;  // records in list order, read contiguously by the render kernels
};

__device__ __forceinline__ void emit_sorted(const TileSortOut& o, uint32_t pos, uint64_t tkey,
                                            uint64_t key) {
  const uint32_t g = (uint32_t)key;
  const uint32_t r = o.pair_rec[g];
  o.keys[pos] = tkey | (key >> 32);
  o.vals[pos] = g;
  o.sorted_rec[pos] = r;
  const float4* src = reinterpret_cast<const float4*>(o.rec + r);
  float4* dst = reinterpret_cast<float4*>(o.lrec + pos);
  const float4 a0 = src[0], a1 = src[1], a2 = src[2], a3 = src[3];
  dst[0] = a0; dst[1] = a1; dst[2] = a2; dst[3] = a3;
}

__device__ __forceinline__ void cmp_swap(uint64_t* k, uint32_t a, uint32_t b, uint32_t n) {
  if (b >= n) return;
  const uint64_t ka = k[a], kb = k[b];
  if (ka > kb) {
    k[a] = kb;
    k[b] = ka;
  }
}

// Sorts k[0, n) ascending (LDS or global memory) with nthreads threads of
// the block; every thread of the block must call it.
__device__ void bitonic_sort(uint64_t* k, uint32_t n, uint32_t tid, uint32_t nthreads) {
  uint32_t m = 1;
  while (m < n) m <<= 1;
  for (uint32_t size = 2; size <= m; size <<= 1) {
    const uint32_t half = size >> 1;
    for (uint32_t idx = tid; idx < m / 2; idx += nthreads) {
      const uint32_t blk = idx / half, off = idx % half;
      cmp_swap(k, blk * size + off, blk * size + size - 1 - off, n);
    }
    __syncthreads();
    for (uint32_t stride = size >> 2; stride > 0; stride >>= 1) {
      for (uint32_t idx = tid; idx < m / 2; idx += nthreads) {
        const uint32_t a = 2 * idx - (idx & (stride - 1));
        cmp_swap(k, a, a + stride, n);
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kWave) k_tile_sort(
    const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ tstart,
    const uint64_t* __restrict__ tile_pre, int T, int32_t* __restrict__ fl,
    const uint64_t* __restrict__ skey, TileSortOut out, uint32_t* __restrict__ ranges,
    uint32_t* __restrict__ long_list, const uint32_t* __restrict__ bstart,
    const uint64_t* __restrict__ bucket_pre, uint32_t* __restrict__ boff,
    const uint32_t* __restrict__ fstart, const uint64_t* __restrict__ full_pre,
    const uint32_t* __restrict__ hstart, const uint64_t* __restrict__ half_pre,
    uint2* __restrict__ bq, int64_t bq_stride) {
  __shared__ uint64_t sk[kTileSortSmall];
  const int t = blockIdx.x;
  const int lane = threadIdx.x;
  const uint64_t P = (uint64_t)fl[F_PAIRS];
  const uint32_t n = fl[F_OVERFLOW] ? 0u : cnt[t];
  const uint64_t start64 = (uint64_t)tstart[t] + tile_pre[t / kScanTile];
  const bool ok = n > 0 && start64 + n <= P;
  if (lane == 0) {
    ranges[2 * (int64_t)t] = ok ? (uint32_t)start64 : 0u;
    ranges[2 * (int64_t)t + 1] = ok ? (uint32_t)(start64 + n) : 0u;
    if (boff) {
      // buckets of 64 positions; a tile without a valid list has none
      boff[t] = bstart[t] + (uint32_t)bucket_pre[t / kScanTile];
      if (t == T - 1) boff[T] = boff[t] + (ok ? (n + kBucket - 1) / kBucket : 0u);
    }
    if (ok && n > kTileSortSmall) long_list[atomicAdd(&fl[F_LONG_TILES], 1)] = (uint32_t)t;
  }
  if (boff && ok) {
    // splat-wise work queues at the scanned positions: the tile's buckets
    // 0 .. full-1 have more than 32 pairs; a last bucket with at most 32
    // goes to the second queue
    uint32_t nb, full, half;
    bucket_split(n, nb, full, half);
    const uint32_t f0 = fstart[t] + (uint32_t)full_pre[t / kScanTile];
    for (uint32_t k = lane; k < full; k += kWave) bq[f0 + k] = make_uint2((uint32_t)t, k);
    if (half && lane == 0)
      bq[bq_stride + hstart[t] + (uint32_t)half_pre[t / kScanTile]] = make_uint2((uint32_t)t, nb - 1);
  }
  if (!ok || n > kTileSortSmall) return;
  const uint32_t start = (uint32_t)start64;
  const uint64_t tkey = (uint64_t)(uint32_t)t << 32;
  if (n <= (uint32_t)kWave) {
    const bool has = (uint32_t)lane < n;
    const uint64_t key = has ? skey[start + lane] : ~0ull;
    uint32_t rank = 0;
    for (uint32_t j = 0; j < n; ++j) {
      const uint64_t kj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(key >> 32), j) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, j);
      rank += kj < key ? 1u : 0u;
    }
    if (has) emit_sorted(out, start + rank, tkey, key);
    return;
  }
  for (uint32_t k = lane; k < n; k += kWave) sk[k] = skey[start + k];
  __syncthreads();
  bitonic_sort(sk, n, lane, kWave);
  for (uint32_t k = lane; k < n; k += kWave) emit_sorted(out, start + k, tkey, sk[k]);
}

__global__ void __launch_bounds__(kLongThreads) k_tile_sort_long(
    const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ tstart,
    const uint64_t* __restrict__ tile_pre, const int32_t* __restrict__ fl,
    const uint32_t* __restrict__ long_list, uint64_t* __restrict__ skey, TileSortOut out) {
  __shared__ uint64_t sk[kTileSortLong];
  const int n_long = fl[F_LONG_TILES];
  for (int li = blockIdx.x; li < n_long; li += gridDim.x) {
    const int t = (int)long_list[li];
    const uint32_t n = cnt[t];
    const uint32_t start = tstart[t] + (uint32_t)tile_pre[t / kScanTile];
    const uint64_t tkey = (uint64_t)(uint32_t)t << 32;
    if (n <= kTileSortLong) {
      for (uint32_t k = threadIdx.x; k < n; k += kLongThreads) sk[k] = skey[start + k];
      __syncthreads();
      bitonic_sort(sk, n, threadIdx.x, kLongThreads);
      for (uint32_t k = threadIdx.x; k < n; k += kLongThreads) emit_sorted(out, start + k, tkey, sk[k]);
    } else {
      bitonic_sort(skey + start, n, threadIdx.x, kLongThreads);
      for (uint32_t k = threadIdx.x; k < n; k += kLongThreads)
        emit_sorted(out, start + k, tkey, skey[start + k]);
    }
    __syncthreads();  // the LDS is reused by the next list
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
  // per-iteration flags 0..10 and the per-tile pair counters
  const int64_t T = P.vt.total_tiles;
  const int64_t m = T > 4 ? T : 4;
  hipLaunchKernelGGL(k_fill2_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                     ws_at<uint32_t>(ws, P.off_flags), (int64_t)11,
                     ws_at<uint32_t>(ws, P.off_tile_cnt), T);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const Plan& P, void* ws, hipStream_t s) {
  int32_t* fl = ws_at<int32_t>(ws, P.off_flags);
  uint32_t* tt = ws_at<uint32_t>(ws, P.off_tt);
  uint32_t* poff = ws_at<uint32_t>(ws, P.off_poff);
  uint64_t* rec_tot = ws_at<uint64_t>(ws, P.off_scan);
  uint64_t* vis_tot = ws_at<uint64_t>(ws, P.off_vis_scan);
  uint32_t* tcnt = ws_at<uint32_t>(ws, P.off_tile_cnt);
  uint32_t* tstart = ws_at<uint32_t>(ws, P.off_tile_start);
  uint64_t* tile_tot = ws_at<uint64_t>(ws, P.off_tile_scan);
  const bool splat = (P.cfg.flags & GS_SPLAT_BWD) != 0;
  uint32_t* bstart = splat ? ws_at<uint32_t>(ws, P.off_bucket_start) : nullptr;
  uint64_t* bucket_tot = splat ? ws_at<uint64_t>(ws, P.off_bucket_scan) : nullptr;
  uint32_t* boff = splat ? ws_at<uint32_t>(ws, P.off_boff) : nullptr;
  const int T = P.vt.total_tiles;
  const int64_t sb = P.scan_blocks, tb = P.tile_scan_blocks;
  uint32_t* fstart = splat ? ws_at<uint32_t>(ws, P.off_full_start) : nullptr;
  uint64_t* full_tot = splat ? ws_at<uint64_t>(ws, P.off_full_scan) : nullptr;
  uint32_t* hstart = splat ? ws_at<uint32_t>(ws, P.off_half_start) : nullptr;
  uint64_t* half_tot = splat ? ws_at<uint64_t>(ws, P.off_half_scan) : nullptr;
  TileScanArgs ta{tcnt, tstart, tile_tot, (int64_t)T, bstart, bucket_tot, fstart, full_tot,
                  hstart, half_tot};
  ScanChannels ch{{rec_tot, vis_tot, tile_tot, bucket_tot, full_tot, half_tot},
                  {sb, sb, tb, tb, tb, tb}, splat ? 6 : 3};
  // at least one block, so that the flags are always set
  hipLaunchKernelGGL(k_scans, dim3((unsigned)std::max<int64_t>(sb + tb, 1)), dim3(kScanThreads), 0,
                     s, tt, poff, rec_tot, ws_at<uint32_t>(ws, P.off_vpre), vis_tot, P.n_rec, sb,
                     ta, ch, P.pair_cap, fl);
  uint64_t* skey = ws_at<uint64_t>(ws, P.off_scatter);
  uint32_t* pair_rec = ws_at<uint32_t>(ws, P.off_pair_rec);
  if (P.n_rec > 0) {
    const int64_t blocks = (P.n_rec + 255) / 256;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, tt, poff, rec_tot,
                       ws_at<ushort4>(ws, P.off_rect), ws_at<Rec>(ws, P.off_rec), P.n, P.n_rec,
                       P.vt, fl, tstart, tile_tot, tcnt, skey, pair_rec,
                       ws_at<uint32_t>(ws, P.off_vpre), vis_tot,
                       ws_at<uint32_t>(ws, P.off_vis_list));
  }
  if (T > 0) {
    TileSortOut out{ws_at<uint64_t>(ws, P.off_keys), ws_at<uint32_t>(ws, P.off_vals),
                    ws_at<uint32_t>(ws, P.off_sorted_rec), pair_rec, ws_at<Rec>(ws, P.off_rec),
                    ws_at<Rec>(ws, P.off_srec)};
    uint32_t* long_list = ws_at<uint32_t>(ws, P.off_long);
    hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)T), dim3(kWave), 0, s, tcnt, tstart, tile_tot,
                       T, fl, skey, out, ws_at<uint32_t>(ws, P.off_ranges), long_list, bstart,
                       bucket_tot, boff, fstart, full_tot, hstart, half_tot,
                       splat ? ws_at<uint2>(ws, P.off_bq) : nullptr, P.ckpt_slots);
    const int long_grid = (int)std::min<int64_t>(T, 256);
    hipLaunchKernelGGL(k_tile_sort_long, dim3((unsigned)long_grid), dim3(kLongThreads), 0, s,
                       tcnt, tstart, tile_tot, fl, long_list, skey, out);
  }
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

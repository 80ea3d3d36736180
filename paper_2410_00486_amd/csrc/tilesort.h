// Per-tile list sort of the binning, shared by the stand-alone tile sort and
// the forward kernel of a whole iteration (which sorts its tile's list
// itself before compositing it).
//
// Output per tile: sorted keys (tile << 32 | depth bits), generation
// indices, record ids, the records in list order, the [start, end) range
// ((0, 0) when empty) and, for the splat-wise backward, the tile's entries
// in the two bucket queues.  Keys are unique, so any correct sort gives the
// same lists.  One wavefront sorts lists up to 64 keys in registers (rank =
// number of smaller keys) and up to kTileSortSmall keys with a bitonic
// network in LDS; longer lists (listed by the binning scan) go to 1024-thread
// blocks, with the same network in LDS up to kTileSortLong keys and in place
// in global memory beyond.  The limit is low on purpose: inside a whole
// iteration the wavefront that sorts a list also composites it, and a
// long list sorted there would hold back the end of the forward (its
// wavefront starts first but finishes last), while the binning sorts the
// few long lists in parallel before the forward starts.  The block's LDS
// holds kTileSortLong keys (64 KB), so that two blocks share a CU and one
// block's barrier waits overlap the other's compares: views with thousands
// of pairs per tile send almost every list here.
//
// The network keeps every merge ascending (the first compare of a merge
// pairs i with its mirror in the block), so positions past the list end act
// as +infinity and are never touched: no padding is written.
#pragma once

#include "gs_internal.h"

namespace gs {

constexpr uint32_t kTileSortSmall = 128;
// lists of kTileSortSmall + 1 .. kTileSortMid pairs: one wavefront each
constexpr uint32_t kTileSortMid = 1024;
constexpr uint32_t kTileSortLong = 8192;
constexpr int kLongThreads = 1024;

// Splits a tile of c pairs into buckets of 64 positions: all but possibly
// the last hold more than 32 pairs (full); a last bucket with at most 32
// pairs is a half bucket.
__device__ __forceinline__ void bucket_split(uint32_t c, uint32_t& nb, uint32_t& full,
                                             uint32_t& half) {
  nb = (c + kBucket - 1) / kBucket;
  const uint32_t r = c - (nb > 0 ? (nb - 1) * kBucket : 0u);  // pairs of the last bucket
  half = (c > 0 && r <= 32) ? 1u : 0u;
  full = nb - half;
}

struct TileSortOut {
  uint64_t* keys;
  uint32_t* vals;
  uint32_t* sorted_rec;
  const uint32_t* pair_rec;
  const Rec* rec;
  Rec* lrec;  // records in list order, read contiguously by the render kernels
};

// Writes the pair of key (depth bits << 32 | generation index) at list
// position pos: sorted key, generation index, record id, record; the record
// also to lds_dst when given.
__device__ __forceinline__ void emit_sorted(const TileSortOut& o, uint32_t pos, uint64_t tkey,
                                            uint64_t key, Rec* lds_dst = nullptr) {
  const uint32_t g = (uint32_t)key;
  const uint32_t r = o.pair_rec[g];
  o.keys[pos] = tkey | (key >> 32);
  o.vals[pos] = g;
  o.sorted_rec[pos] = r;
  const float4* src = reinterpret_cast<const float4*>(o.rec + r);
  float4* dst = reinterpret_cast<float4*>(o.lrec + pos);
  const float4 a0 = src[0], a1 = src[1], a2 = src[2], a3 = src[3];
  dst[0] = a0; dst[1] = a1; dst[2] = a2; dst[3] = a3;
  if (lds_dst) {
    float4* l = reinterpret_cast<float4*>(lds_dst);
    l[0] = a0; l[1] = a1; l[2] = a2; l[3] = a3;
  }
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
__device__ inline void bitonic_sort(uint64_t* k, uint32_t n, uint32_t tid, uint32_t nthreads) {
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

// Sorts k[0, n) ascending in LDS with the 64 lanes of one wavefront and
// wavefront-level syncs only (the other wavefronts of its workgroup sort
// their own lists meanwhile).
__device__ inline void bitonic_sort_wave(uint64_t* k, uint32_t n, uint32_t lane) {
  uint32_t m = 1;
  while (m < n) m <<= 1;
  for (uint32_t size = 2; size <= m; size <<= 1) {
    const uint32_t half = size >> 1;
    for (uint32_t idx = lane; idx < m / 2; idx += kWave) {
      const uint32_t blk = idx / half, off = idx % half;
      cmp_swap(k, blk * size + off, blk * size + size - 1 - off, n);
    }
    wave_lds_sync();
    for (uint32_t stride = size >> 2; stride > 0; stride >>= 1) {
      for (uint32_t idx = lane; idx < m / 2; idx += kWave) {
        const uint32_t a = 2 * idx - (idx & (stride - 1));
        cmp_swap(k, a, a + stride, n);
      }
      wave_lds_sync();
    }
  }
}

// Everything a wavefront needs to sort one tile's list.
struct TileSortArgs {
  uint32_t* cnt;           // pairs per tile (the scatter's cursors); cleared after use
  const uint32_t* tstart;  // list start per tile
  const int32_t* fl;
  const uint64_t* skey;    // scattered keys (depth bits << 32 | generation index)
  TileSortOut out;
  uint32_t* ranges;
  const uint32_t* fstart;  // splat-wise only (bq non-null): queue positions
  const uint32_t* hstart;
  uint2* bq;
  int64_t bq_stride;
  // the long-list kernel runs after this one (it then clears the counters of
  // the long lists itself) rather than before
  bool long_after;
  // the lists were sorted by the radix binning: ranges, queue entries and
  // counter clears only
  bool presorted;
};

// What a wavefront that sorted a tile knows about its list: the range
// ((0, 0) when empty), whether this wavefront wrote the sorted records (then
// a read of them inside the same kernel must not be served by the vector L1,
// which may hold an older copy of the line), and whether its first
// stage_cap records are also in the staging LDS already.
struct TileList {
  uint32_t start, end;
  bool fresh, staged;
};

// One wavefront (lane = lane of a single-wave workgroup): range and bucket
// queue entries of tile t, then, for a list of at most kTileSortSmall pairs,
// the sort and the sorted outputs.  sk: kTileSortSmall keys of LDS.
// Longer lists are left to the long-list kernel.  stage (optional, at least
// stage_cap records of LDS, may alias sk): the list's first stage_cap
// records also land there in list order (all of a list of at most 64 pairs
// only if it fits).
__device__ inline TileList sort_tile_wave(const TileSortArgs& A, int t, int lane, uint64_t* sk,
                                          Rec* stage = nullptr, int stage_cap = 0) {
  const uint64_t P = (uint64_t)A.fl[F_PAIRS];
  const uint32_t c = A.cnt[t];
  const uint32_t n = A.fl[F_OVERFLOW] ? 0u : c;
  const uint64_t start64 = A.tstart[t];
  const bool ok = n > 0 && start64 + n <= P;
  if (lane == 0) {
    A.ranges[2 * (int64_t)t] = ok ? (uint32_t)start64 : 0u;
    A.ranges[2 * (int64_t)t + 1] = ok ? (uint32_t)(start64 + n) : 0u;
    // the counter is consumed: zero again for the next projection (a long
    // list's counter is still read by a long-list kernel that runs after)
    if (!(A.long_after && c > kTileSortSmall)) A.cnt[t] = 0u;
  }
  if (A.bq && ok) {
    // splat-wise work queues at the scanned positions: the tile's buckets
    // 0 .. full-1 have more than 32 pairs; a last bucket with at most 32
    // goes to the second queue
    uint32_t nb, full, half;
    bucket_split(n, nb, full, half);
    const uint32_t f0 = A.fstart[t];
    for (uint32_t k = lane; k < full; k += kWave) A.bq[f0 + k] = make_uint2((uint32_t)t, k);
    if (half && lane == 0) A.bq[A.bq_stride + A.hstart[t]] = make_uint2((uint32_t)t, nb - 1);
  }
  TileList L{ok ? (uint32_t)start64 : 0u, ok ? (uint32_t)(start64 + n) : 0u, false, false};
  if (!ok || n > kTileSortSmall || A.presorted) return L;  // uniform
  L.fresh = true;
  const uint32_t start = (uint32_t)start64;
  const uint64_t tkey = (uint64_t)(uint32_t)t << 32;
  if (n <= (uint32_t)kWave) {
    const bool has = (uint32_t)lane < n;
    const uint64_t key = has ? A.skey[start + lane] : ~0ull;
    uint32_t rank = 0;
    for (uint32_t j = 0; j < n; ++j) {
      const uint64_t kj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(key >> 32), j) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, j);
      rank += kj < key ? 1u : 0u;
    }
    L.staged = stage && n <= (uint32_t)stage_cap;
    if (has) emit_sorted(A.out, start + rank, tkey, key, L.staged ? stage + rank : nullptr);
    return L;
  }
  for (uint32_t k = lane; k < n; k += kWave) sk[k] = A.skey[start + k];
  __syncthreads();
  bitonic_sort(sk, n, lane, kWave);
  // The lane's sorted keys are written out and their record ids looked up
  // all at once (one memory round trip for all of them instead of one per
  // position); the ids then wait in the keys' LDS for the record gathers.
  constexpr int KMAX = kTileSortSmall / kWave;
  const TileSortOut& o = A.out;
  uint32_t r[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const uint32_t k = (uint32_t)lane + (uint32_t)q * kWave;
    r[q] = 0u;
    if (k < n) {
      const uint64_t key = sk[k];
      const uint32_t g = (uint32_t)key;
      o.keys[start + k] = tkey | (key >> 32);
      o.vals[start + k] = g;
      r[q] = o.pair_rec[g];
    }
  }
  __syncthreads();  // every key has been read
  uint32_t* sr = reinterpret_cast<uint32_t*>(sk);
#pragma unroll
  for (int q = 0; q < KMAX; ++q) {
    const uint32_t k = (uint32_t)lane + (uint32_t)q * kWave;
    if (k < n) sr[k] = r[q];
  }
  for (uint32_t k = lane; k < n; k += kWave) {  // this lane's own positions
    const uint32_t rk = sr[k];
    o.sorted_rec[start + k] = rk;
    const float4* src = reinterpret_cast<const float4*>(o.rec + rk);
    float4* dst = reinterpret_cast<float4*>(o.lrec + start + k);
    const float4 a0 = src[0], a1 = src[1], a2 = src[2], a3 = src[3];
    dst[0] = a0; dst[1] = a1; dst[2] = a2; dst[3] = a3;
  }
  return L;
}

}  // namespace gs

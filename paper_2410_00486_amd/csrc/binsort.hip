// a2: tile binning.  Pairs are the (Gaussian, tile) incidences of the exact
// tile boxes, numbered in generation order (record-major, row-major tiles
// within a box).  The order the renderer needs is (tile, depth, generation
// index): unique, so the result is bit-exact whatever the schedule.
//
// The projection counts pairs per tile and per chunk of 64 Gaussians as it
// computes the boxes.  Then: one block scans the chunk counts (generation
// offsets, visible-list positions) and the tile counts (list starts, bucket
// offsets and queue positions); one scatter puts every pair into its tile's
// list at an atomically taken slot with the key (depth bits << 32 |
// generation index); a per-tile sort orders those keys (one wavefront per
// tile: ranks in registers up to 64 keys, a bitonic network in LDS up to
// 128; longer lists go to 1024-thread blocks, in LDS up to 8192 keys and in
// global memory beyond).  Four launches whatever the pair count, no
// spin-waits; graph-capturable.
//
// The scan block also writes the work order of the render kernels: tiles
// with long lists first.  The general stable LSD
// radix sort (8-bit digits, wave64 ballot ranking) below serves the
// standalone key/value sort.
#include "tilesort.h"
#include "wavescan.h"

namespace gs {
namespace {

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void k_set_i32(int32_t* __restrict__ p, int32_t value) { *p = value; }

// Clears a[0, na) and b[0, nb).
__global__ void k_fill2_u32(uint32_t* __restrict__ a, int64_t na, uint32_t* __restrict__ b,
                            int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) a[i] = 0u;
  if (i < nb) b[i] = 0u;
}

// ---------------------------------------------------------------- scans
// The projection writes, for every chunk of 64 Gaussians of a view (one
// wavefront), its pair count and its number of visible records; and the
// pair count of every tile.  One block scans both: chunks -> generation
// offset and visible-list position of the chunk's first record; tiles ->
// list start, bucket offset and positions in the two splat-wise bucket
// queues.  One block needs no inter-block handshake (a grid-wide fence
// costs more than the scan itself at these sizes), and the results are
// absolute, so the consumers add nothing.
//
// Offsets are stored as u32, exact whenever the pair total fits the pair
// capacity (< 2^31); otherwise the overflow flag stops every consumer.  The
// running sums are 64-bit.

constexpr int kScanBlock = 1024;  // threads of the scan block
constexpr int kScanVec = 2;       // uint4 loads per thread and array in a round
// A round: 4 * kScanVec consecutive tiles and 2 * kScanVec consecutive
// chunks per thread, loaded and stored as uint4.
constexpr int64_t kTileRound = (int64_t)kScanBlock * 4 * kScanVec;
constexpr int64_t kChunkRound = (int64_t)kScanBlock * 2 * kScanVec;

struct ScanArgs {
  const uint2* chunk_cnt;  // (pairs, visible records) per chunk
  uint2* chunk_pre;        // (generation offset, visible-list position) per chunk
  int64_t n_chunks;
  uint32_t* cnt;           // pairs per tile; cleared here (the scatter's cursors)
  uint32_t* tstart;        // list start per tile
  int64_t n_tiles;
  uint32_t* boff;          // splat-wise only (else null): bucket offset per tile, [T] = total
  uint32_t* fstart;        // position of the tile's first full bucket in queue 0
  uint32_t* hstart;        // position of the tile's half bucket in queue 1
  uint32_t* order;         // work order of the render kernels, longest tiles first
  uint4* long_list;        // (tile, list start, pairs, -) of the lists for the long-list sort
  // kScanBoth: chunks and tile counts (the projection's); kScanChunks: the
  // chunks alone (radix binning, before the pairs exist); kScanTiles: the
  // tiles alone from the list ends (cnt) and starts (tstart) that the radix
  // binning found in its sorted keys, with the counts written back to cnt
  int mode;
};
constexpr int kScanBoth = 0, kScanChunks = 1, kScanTiles = 2;

// Work order of the render kernels: tiles with at least kLongTile pairs
// first (in tile order), then the others (in reverse tile order), so that
// the long lists start in the first round of the dispatch and the tail is
// made of short ones.  Both positions come out of the scan.
constexpr uint32_t kLongTile = 32;

// Block-wide exclusive scan of N64 64-bit and N32 32-bit per-thread sums
// (replaced by the thread's start); the carries (uniform) are added and
// advanced by the block totals.  The 64-bit channels count pairs (their
// totals decide the overflow); the 32-bit ones are exact whenever those fit
// the pair capacity.  w64 / w32 hold (NW + 1) entries per channel.  Every
// thread of the block must call.
template <int N64, int N32>
__device__ __forceinline__ void block_exscan(uint64_t (&s64)[N64], uint32_t (&s32)[N32],
                                             uint64_t (&c64)[N64], uint32_t (&c32)[N32],
                                             uint64_t* w64, uint32_t* w32) {
  constexpr int NW = kScanBlock / kWave;
  static_assert(NW == 16, "the wave sums are scanned within one 16-lane row");
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint64_t i64[N64];
  uint32_t i32[N32];
#pragma unroll
  for (int c = 0; c < N64; ++c) i64[c] = scan_dpp<6>(s64[c]);
#pragma unroll
  for (int c = 0; c < N32; ++c) i32[c] = scan_dpp<6>(s32[c]);
  if (lane == kWave - 1) {
#pragma unroll
    for (int c = 0; c < N64; ++c) w64[c * (NW + 1) + w] = i64[c];
#pragma unroll
    for (int c = 0; c < N32; ++c) w32[c * (NW + 1) + w] = i32[c];
  }
  __syncthreads();
  if (w == 0) {
    // lanes 0..15 of wave 0 scan the wave sums: exclusive offsets (plus the
    // carry) at [0, NW), the new carry at [NW]
#pragma unroll
    for (int c = 0; c < N64; ++c) {
      const uint64_t x = lane < NW ? w64[c * (NW + 1) + lane] : 0ull;
      const uint64_t j = scan_dpp<4>(x);
      if (lane < NW) w64[c * (NW + 1) + lane] = c64[c] + j - x;
      if (lane == NW - 1) w64[c * (NW + 1) + NW] = c64[c] + j;
    }
#pragma unroll
    for (int c = 0; c < N32; ++c) {
      const uint32_t x = lane < NW ? w32[c * (NW + 1) + lane] : 0u;
      const uint32_t j = scan_dpp<4>(x);
      if (lane < NW) w32[c * (NW + 1) + lane] = c32[c] + j - x;
      if (lane == NW - 1) w32[c * (NW + 1) + NW] = c32[c] + j;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < N64; ++c) {
    s64[c] = w64[c * (NW + 1) + w] + i64[c] - s64[c];
    c64[c] = w64[c * (NW + 1) + NW];
  }
#pragma unroll
  for (int c = 0; c < N32; ++c) {
    s32[c] = w32[c * (NW + 1) + w] + i32[c] - s32[c];
    c32[c] = w32[c * (NW + 1) + NW];
  }
  __syncthreads();  // the wave sums are rewritten by the next round
}

// Four consecutive u32 from a[i], zeros past n (a is 16-byte aligned, i a
// multiple of 4).
__device__ __forceinline__ uint4 load4(const uint32_t* __restrict__ a, int64_t i, int64_t n) {
  if (i + 4 <= n) return *reinterpret_cast<const uint4*>(a + i);
  uint4 x = make_uint4(0u, 0u, 0u, 0u);
  if (i < n) x.x = a[i];
  if (i + 1 < n) x.y = a[i + 1];
  if (i + 2 < n) x.z = a[i + 2];
  return x;
}

__device__ __forceinline__ void store4(uint32_t* __restrict__ a, int64_t i, int64_t n, uint4 x) {
  if (i + 4 <= n) {
    *reinterpret_cast<uint4*>(a + i) = x;
    return;
  }
  if (i < n) a[i] = x.x;
  if (i + 1 < n) a[i + 1] = x.y;
  if (i + 2 < n) a[i + 2] = x.z;
}

// Per-thread inputs of one round: 4 * kScanVec tiles and 2 * kScanVec
// chunks, and the thread's sums over them.  Channels: 64-bit tile pairs and
// chunk pairs; 32-bit buckets, half buckets, visible records, tiles with at
// least kLongTile pairs (work order), lists longer than kTileSortSmall
// (long-list sort).
constexpr int kScanN32 = 5;
struct ScanRound {
  static constexpr int NT = 4 * kScanVec, NC = 2 * kScanVec;
  int64_t it, ic;  // first tile and first chunk of the thread
  uint32_t tc[NT], nb[NT], h[NT], cp[NC], cv[NC];
  uint64_t s64[2];
  uint32_t s32[kScanN32];
};

__device__ __forceinline__ void scan_load(const ScanArgs& A, int64_t r, ScanRound& R) {
  const int64_t T = A.n_tiles, C = A.n_chunks;
  R.it = r * kTileRound + (int64_t)ScanRound::NT * threadIdx.x;
  R.ic = r * kChunkRound + (int64_t)ScanRound::NC * threadIdx.x;
  const uint32_t* chunk_in = reinterpret_cast<const uint32_t*>(A.chunk_cnt);
#pragma unroll
  for (int k = 0; k < kScanVec; ++k) {
    uint4 x = load4(A.cnt, R.it + 4 * k, T);
    if (A.mode == kScanTiles) {  // list end (0: no pairs) minus list start
      const uint4 st = load4(A.tstart, R.it + 4 * k, T);
      x = make_uint4(x.x ? x.x - st.x : 0u, x.y ? x.y - st.y : 0u, x.z ? x.z - st.z : 0u,
                     x.w ? x.w - st.w : 0u);
    }
    R.tc[4 * k] = x.x; R.tc[4 * k + 1] = x.y; R.tc[4 * k + 2] = x.z; R.tc[4 * k + 3] = x.w;
    const uint4 y = load4(chunk_in, 2 * (R.ic + 2 * k), 2 * C);
    R.cp[2 * k] = y.x; R.cv[2 * k] = y.y; R.cp[2 * k + 1] = y.z; R.cv[2 * k + 1] = y.w;
  }
  R.s64[0] = R.s64[1] = 0;
#pragma unroll
  for (int c = 0; c < kScanN32; ++c) R.s32[c] = 0;
#pragma unroll
  for (int k = 0; k < ScanRound::NT; ++k) {
    uint32_t f;
    bucket_split(R.tc[k], R.nb[k], f, R.h[k]);
    R.s64[0] += R.tc[k];
    R.s32[0] += R.nb[k];
    R.s32[1] += R.h[k];
    R.s32[3] += R.tc[k] >= kLongTile ? 1u : 0u;
    R.s32[4] += R.tc[k] > kTileSortSmall ? 1u : 0u;
  }
#pragma unroll
  for (int k = 0; k < ScanRound::NC; ++k) {
    R.s64[1] += R.cp[k];
    R.s32[2] += R.cv[k];
  }
}

// Writes the round's outputs from the thread's exclusive starts (R.s64 /
// R.s32 after the block scan): list starts, bucket offsets and queue
// positions, work order, long-list entries (in tile order), chunk offsets;
// and clears the tile counters (the scatter's cursors).
__device__ __forceinline__ void scan_emit(const ScanArgs& A, ScanRound& R) {
  const int64_t T = A.n_tiles, C = A.n_chunks;
  uint32_t* chunk_out = reinterpret_cast<uint32_t*>(A.chunk_pre);
#pragma unroll
  for (int k = 0; k < kScanVec; ++k) {
    uint32_t ts[4], bs[4], hs[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t t = R.it + 4 * k + e;
      const uint32_t c = R.tc[4 * k + e];
      // work order: long tiles from the front, the others from the back
      // (both positions follow from the long tiles before t)
      if (t < T)
        A.order[c >= kLongTile ? R.s32[3] : (uint32_t)(T - 1 - (t - R.s32[3]))] = (uint32_t)t;
      // lists too long for one wavefront: listed for the long-list sort
      if (t < T && c > kTileSortSmall)
        A.long_list[R.s32[4]] = make_uint4((uint32_t)t, (uint32_t)R.s64[0], c, 0u);
      ts[e] = (uint32_t)R.s64[0];
      bs[e] = R.s32[0];
      hs[e] = R.s32[1];
      R.s64[0] += c;
      R.s32[0] += R.nb[4 * k + e];
      R.s32[1] += R.h[4 * k + e];
      R.s32[3] += c >= kLongTile ? 1u : 0u;
      R.s32[4] += c > kTileSortSmall ? 1u : 0u;
    }
    store4(A.tstart, R.it + 4 * k, T, make_uint4(ts[0], ts[1], ts[2], ts[3]));
    // the scatter's cursors start at zero; the radix binning's per-tile
    // pass reads the counts
    store4(A.cnt, R.it + 4 * k, T,
           A.mode == kScanTiles ? make_uint4(R.tc[4 * k], R.tc[4 * k + 1], R.tc[4 * k + 2],
                                             R.tc[4 * k + 3])
                                : make_uint4(0u, 0u, 0u, 0u));
    if (A.boff) {
      store4(A.boff, R.it + 4 * k, T, make_uint4(bs[0], bs[1], bs[2], bs[3]));
      store4(A.fstart, R.it + 4 * k, T,
             make_uint4(bs[0] - hs[0], bs[1] - hs[1], bs[2] - hs[2], bs[3] - hs[3]));
      store4(A.hstart, R.it + 4 * k, T, make_uint4(hs[0], hs[1], hs[2], hs[3]));
    }
    const uint32_t p0 = (uint32_t)R.s64[1], v0 = R.s32[2];
    const uint32_t p1 = p0 + R.cp[2 * k], v1 = v0 + R.cv[2 * k];
    store4(chunk_out, 2 * (R.ic + 2 * k), 2 * C, make_uint4(p0, v0, p1, v1));
    R.s64[1] = p1 + R.cp[2 * k + 1];
    R.s32[2] = v1 + R.cv[2 * k + 1];
  }
}

// Totals -> flags (one thread).  Both pair totals count the same pairs; a
// mismatch is reported as an overflow so that nothing is scattered.
__device__ __forceinline__ void scan_finish(const ScanArgs& A, const uint64_t (&c64)[2],
                                            const uint32_t (&c32)[kScanN32], int64_t cap,
                                            int32_t* __restrict__ fl, const StepAdvance& st) {
  const bool splat = A.boff != nullptr;
  if (A.mode == kScanTiles) {
    // the pair totals were settled by the chunk scan before
    const bool over = fl[F_OVERFLOW] != 0;
    fl[F_LONG_TILES] = over ? 0 : (int32_t)c32[4];
    fl[F_BQ_FULL] = (over || !splat) ? 0 : (int32_t)(c32[0] - c32[1]);
    fl[F_BQ_HALF] = (over || !splat) ? 0 : (int32_t)c32[1];
    if (splat) A.boff[A.n_tiles] = c32[0];
    return;
  }
  const uint64_t tile_pairs = c64[0], chunk_pairs = c64[1];
  const bool chunks_only = A.mode == kScanChunks;
  const uint64_t pairs = chunks_only ? chunk_pairs : tile_pairs;
  const bool over = pairs > (uint64_t)cap || (!chunks_only && tile_pairs != chunk_pairs);
  fl[F_OVERFLOW] = over ? 1 : 0;
  fl[F_PAIRS] = over ? 0 : (int32_t)pairs;
  fl[F_PAIRS_WANTED] = pairs > 0x7FFFFFFFull ? 0x7FFFFFFF : (int32_t)pairs;
  fl[F_VISIBLE] = (int32_t)c32[2];
  fl[F_NONFINITE] = fl[F_NF_ACC];  // counted by the projection
  fl[F_NF_ACC] = 0;
  if (!chunks_only) {
    // the bucket queues are filled by the tile sort at the positions scanned
    // here; the long lists are sorted by their own kernel (none on overflow)
    fl[F_LONG_TILES] = (int32_t)c32[4];
    fl[F_BQ_FULL] = (over || !splat) ? 0 : (int32_t)(c32[0] - c32[1]);
    fl[F_BQ_HALF] = (over || !splat) ? 0 : (int32_t)c32[1];
    if (splat) A.boff[A.n_tiles] = c32[0];
  }
  // a whole iteration with Adam advances its step here, once the pairs are
  // known to fit: after an overflow the iteration's Adam launch changes
  // nothing, and neither does the step counter
  if (st.step && !over) advance_step(st);
}

// One block, all rounds in sequence (small plans: no extra launches).
__global__ void __launch_bounds__(kScanBlock) k_scans(ScanArgs A, int64_t cap,
                                                      int32_t* __restrict__ fl, StepAdvance st) {
  constexpr int NW = kScanBlock / kWave;
  __shared__ uint64_t w64[2 * (NW + 1)];
  __shared__ uint32_t w32[kScanN32 * (NW + 1)];
  uint64_t c64[2] = {0, 0};
  uint32_t c32[kScanN32] = {0, 0, 0, 0, 0};
  const int64_t rt = (A.n_tiles + kTileRound - 1) / kTileRound;
  const int64_t rc = (A.n_chunks + kChunkRound - 1) / kChunkRound;
  const int64_t rounds = rt > rc ? rt : rc;
  for (int64_t r = 0; r < rounds; ++r) {
    ScanRound R;
    scan_load(A, r, R);
    block_exscan<2, kScanN32>(R.s64, R.s32, c64, c32, w64, w32);
    scan_emit(A, R);
  }
  if (threadIdx.x == 0) scan_finish(A, c64, c32, cap, fl, st);
}

// Larger plans: one block per round in three launches.  Per-round totals of
// every channel (reduce), their exclusive scan and the flags (top, one
// block), then every round again from its carry (down).
struct ScanPart {
  uint64_t p64[2];
  uint32_t p32[kScanN32];
  uint32_t pad;
};

__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(ScanArgs A,
                                                            ScanPart* __restrict__ part) {
  constexpr int NW = kScanBlock / kWave;
  __shared__ uint64_t w64[2 * (NW + 1)];
  __shared__ uint32_t w32[kScanN32 * (NW + 1)];
  uint64_t c64[2] = {0, 0};
  uint32_t c32[kScanN32] = {0, 0, 0, 0, 0};
  ScanRound R;
  scan_load(A, blockIdx.x, R);
  block_exscan<2, kScanN32>(R.s64, R.s32, c64, c32, w64, w32);  // c64 / c32: block totals
  if (threadIdx.x == 0) {
    ScanPart p;
    p.p64[0] = c64[0];
    p.p64[1] = c64[1];
#pragma unroll
    for (int c = 0; c < kScanN32; ++c) p.p32[c] = c32[c];
    p.pad = 0u;
    part[blockIdx.x] = p;
  }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_top(ScanArgs A, ScanPart* __restrict__ part,
                                                         int64_t n_parts, int64_t cap,
                                                         int32_t* __restrict__ fl, StepAdvance st) {
  constexpr int NW = kScanBlock / kWave;
  __shared__ uint64_t w64[2 * (NW + 1)];
  __shared__ uint32_t w32[kScanN32 * (NW + 1)];
  uint64_t c64[2] = {0, 0};
  uint32_t c32[kScanN32] = {0, 0, 0, 0, 0};
  for (int64_t base = 0; base < n_parts; base += kScanBlock) {
    const int64_t i = base + threadIdx.x;
    uint64_t s64[2] = {0, 0};
    uint32_t s32[kScanN32] = {0, 0, 0, 0, 0};
    if (i < n_parts) {
      const ScanPart p = part[i];
      s64[0] = p.p64[0];
      s64[1] = p.p64[1];
#pragma unroll
      for (int c = 0; c < kScanN32; ++c) s32[c] = p.p32[c];
    }
    block_exscan<2, kScanN32>(s64, s32, c64, c32, w64, w32);
    if (i < n_parts) {
      ScanPart p;
      p.p64[0] = s64[0];
      p.p64[1] = s64[1];
#pragma unroll
      for (int c = 0; c < kScanN32; ++c) p.p32[c] = s32[c];
      p.pad = 0u;
      part[i] = p;
    }
  }
  if (threadIdx.x == 0) scan_finish(A, c64, c32, cap, fl, st);
}

__global__ void __launch_bounds__(kScanBlock) k_scan_down(ScanArgs A,
                                                          const ScanPart* __restrict__ part) {
  constexpr int NW = kScanBlock / kWave;
  __shared__ uint64_t w64[2 * (NW + 1)];
  __shared__ uint32_t w32[kScanN32 * (NW + 1)];
  const ScanPart p = part[blockIdx.x];  // exclusive carry of this round
  uint64_t c64[2] = {p.p64[0], p.p64[1]};
  uint32_t c32[kScanN32];
#pragma unroll
  for (int c = 0; c < kScanN32; ++c) c32[c] = p.p32[c];
  ScanRound R;
  scan_load(A, blockIdx.x, R);
  block_exscan<2, kScanN32>(R.s64, R.s32, c64, c32, w64, w32);
  scan_emit(A, R);
}

// ---------------------------------------------------------------- scatter
// One wavefront per chunk (64 Gaussians of one view, the projection's
// wavefront): the generation offsets of its records become absolute (poff),
// its visible records are listed in index order, and every pair gets the
// next free slot of its tile's list with key (depth bits << 32 | generation
// index); pair -> record is recorded.  The chunk's pairs are spread evenly
// over the lanes (exclusive scan of the pair counts, binary search of a
// pair's record in LDS), so a large Gaussian does not serialise its tiles'
// slot claims on one lane.
__global__ void __launch_bounds__(256) k_scatter(
    const uint32_t* __restrict__ tt, uint32_t* __restrict__ poff,
    const uint2* __restrict__ chunk_pre, int64_t chunks_per_view, int64_t n_chunks,
    const ushort4* __restrict__ rect, const Rec* __restrict__ rec, int64_t n, ViewTable vt,
    const int32_t* __restrict__ fl, const uint32_t* __restrict__ tstart,
    uint32_t* __restrict__ cursor, uint64_t* __restrict__ skey, uint32_t* __restrict__ pair_rec,
    uint32_t* __restrict__ vis_list, uint32_t* __restrict__ vis_clamp) {
  constexpr int NW = 256 / kWave;
  __shared__ uint32_t s_pre[NW][kWave];
  __shared__ uint32_t s_p0[NW][kWave], s_dbits[NW][kWave], s_x0y0[NW][kWave];
  __shared__ uint32_t s_tile0[NW][kWave];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = lane_id();
  const int64_t gw = (int64_t)blockIdx.x * NW + w;  // chunk
  if (gw >= n_chunks) return;                       // whole wavefront; no block barrier below
  const int v = (int)(gw / chunks_per_view);
  const int64_t gi = (gw - (int64_t)v * chunks_per_view) * kWave + lane;  // Gaussian
  const int64_t ri = (int64_t)v * n + gi;                                 // record
  const uint64_t P = (uint64_t)fl[F_PAIRS];
  const bool over = fl[F_OVERFLOW] != 0;
  const uint32_t c = (gi < n && !over) ? tt[ri] : 0u;
  const uint2 cp = chunk_pre[gw];
  // the record's tile box and depth are fetched before the scan of the
  // counts, which then runs while they are in flight (DPP, no LDS)
  ushort4 r = make_ushort4(0, 0, 0, 0);
  uint32_t dbits = 0, cbits = 0;
  if (c > 0) {
    r = rect[ri];
    dbits = __float_as_uint(rec[ri].z);
    cbits = rec[ri].clamp;  // (same line as the depth)
  }
  const uint32_t incl = scan_dpp<6>(c);
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
  const uint64_t base64 = (uint64_t)cp.x + (incl - c);
  if ((uint64_t)cp.x + total > P) return;  // cannot happen without overflow (uniform)
  const uint64_t vmask = ballot64(c > 0);
  uint32_t p0 = 0, x0y0 = 0, tile0 = 0;
  if (c > 0) {
    p0 = (uint32_t)base64;
    poff[ri] = p0;
    const uint32_t vp = cp.y + (uint32_t)__popcll(vmask & lanemask_lt());
    vis_list[vp] = (uint32_t)ri;
    vis_clamp[vp] = cbits;
    x0y0 = (uint32_t)r.x | ((uint32_t)r.y << 16);
    tile0 = (uint32_t)(r.z - r.x);  // box width in tiles
  }
  if (total == 0) return;
  s_pre[w][lane] = incl - c;
  s_p0[w][lane] = p0;
  s_dbits[w][lane] = dbits;
  s_x0y0[w][lane] = x0y0;
  s_tile0[w][lane] = tile0;
  wave_lds_sync();
  const ViewInfo vi = vt.v[v];
  const uint32_t rec0 = (uint32_t)(ri - lane);
  for (uint32_t q = (uint32_t)lane; q < total; q += kWave) {
    // owner: the last lane whose prefix is <= q (it has pairs)
    int lo = 0, hi = kWave - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[w][mid] <= q) lo = mid; else hi = mid - 1;
    }
    const uint32_t k = q - s_pre[w][lo];
    const uint32_t bw = s_tile0[w][lo], xy = s_x0y0[w][lo];
    const int x = (int)(xy & 0xFFFFu) + (int)(k % bw);
    const int y = (int)(xy >> 16) + (int)(k / bw);
    const int t = vi.tile_off + y * vi.tiles_x + x;
    const uint32_t p = s_p0[w][lo] + k;
    const uint64_t slot = (uint64_t)tstart[t] + atomicAdd(&cursor[t], 1u);
    if (slot < P) skey[slot] = ((uint64_t)s_dbits[w][lo] << 32) | p;
    pair_rec[p] = rec0 + (uint32_t)lo;
  }
}

// ---------------------------------------------------------------- tile sort
// (per-tile sort helpers in tilesort.h)

__global__ void __launch_bounds__(kWave) k_tile_sort(TileSortArgs A) {
  __shared__ uint64_t sk[kTileSortSmall];
  (void)sort_tile_wave(A, blockIdx.x, threadIdx.x, sk);
}

// Lists of kTileSortSmall + 1 .. kTileSortMid pairs: one wavefront per list
// (four per workgroup, each with its own LDS), bitonic network with
// wavefront-level syncs, then the sorted outputs with the record ids of all
// of a lane's positions looked up in one round trip.
constexpr int kMidWaves = 4;
__global__ void __launch_bounds__(kMidWaves * kWave) k_tile_sort_mid(
    uint32_t* __restrict__ cnt, const int32_t* __restrict__ fl, const uint4* __restrict__ long_list,
    const uint64_t* __restrict__ skey, TileSortOut out, int clear) {
  __shared__ uint64_t sk_all[kMidWaves][kTileSortMid];
  const int w = threadIdx.x / kWave, lane = lane_id();
  uint64_t* sk = sk_all[w];
  const int n_long = fl[F_OVERFLOW] ? 0 : fl[F_LONG_TILES];
  constexpr int KMAX = kTileSortMid / kWave;
  for (int li = blockIdx.x * kMidWaves + w; li < n_long; li += gridDim.x * kMidWaves) {
    const uint4 e = long_list[li];  // (tile, list start, pairs, -)
    const uint32_t n = e.z;
    if (n > kTileSortMid) continue;  // uniform: the long-list kernel's
    const int t = (int)e.x;
    const uint32_t start = e.y;
    const uint64_t tkey = (uint64_t)(uint32_t)t << 32;
    for (uint32_t k = lane; k < n; k += kWave) sk[k] = skey[start + k];
    wave_lds_sync();
    bitonic_sort_wave(sk, n, (uint32_t)lane);
    uint32_t r[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const uint32_t k = (uint32_t)lane + (uint32_t)q * kWave;
      r[q] = 0u;
      if (k < n) {
        const uint64_t key = sk[k];
        const uint32_t g = (uint32_t)key;
        out.keys[start + k] = tkey | (key >> 32);
        out.vals[start + k] = g;
        r[q] = out.pair_rec[g];
      }
    }
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      const uint32_t k = (uint32_t)lane + (uint32_t)q * kWave;
      if (k < n) {
        const uint32_t rk = r[q];
        out.sorted_rec[start + k] = rk;
        const float4* src = reinterpret_cast<const float4*>(out.rec + rk);
        float4* dst = reinterpret_cast<float4*>(out.lrec + start + k);
        const float4 a0 = src[0], a1 = src[1], a2 = src[2], a3 = src[3];
        dst[0] = a0; dst[1] = a1; dst[2] = a2; dst[3] = a3;
      }
    }
    wave_lds_sync();  // every key read before the next list overwrites them
    // counter consumed (when the per-tile pass ran before this kernel)
    if (clear && lane == 0) cnt[t] = 0u;
  }
}

__global__ void __launch_bounds__(kLongThreads) k_tile_sort_long(
    uint32_t* __restrict__ cnt, const int32_t* __restrict__ fl, const uint4* __restrict__ long_list,
    uint64_t* __restrict__ skey, TileSortOut out, int clear) {
  __shared__ uint64_t sk[kTileSortLong];
  const int n_long = fl[F_OVERFLOW] ? 0 : fl[F_LONG_TILES];
  for (int li = blockIdx.x; li < n_long; li += gridDim.x) {
    const uint4 e = long_list[li];  // the scan recorded the list's start and length
    const int t = (int)e.x;
    const uint32_t start = e.y, n = e.z;
    if (n <= kTileSortMid) continue;  // uniform: sorted by k_tile_sort_mid
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
    // counter consumed (when the per-tile pass ran before this kernel)
    if (clear && threadIdx.x == 0) cnt[t] = 0u;
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

hipError_t launch_rb_generate(const Plan& P, void* ws, hipStream_t s);
hipError_t launch_rb_tile_sort(const Plan& P, void* ws, hipStream_t s);
hipError_t launch_rb_runs(const Plan& P, void* ws, hipStream_t s);

hipError_t launch_set_i32(int32_t* p, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_clear_counters(const Plan& P, void* ws, hipStream_t s) {
  // per-iteration flags 0..10 and the per-tile pair counters
  const int64_t T = P.vt.total_tiles;
  const int64_t m = T > 4 ? T : 4;
  hipLaunchKernelGGL(k_fill2_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                     ws_at<uint32_t>(ws, P.off_flags), (int64_t)(F_NF_ACC + 1),
                     ws_at<uint32_t>(ws, P.off_tile_cnt), T);
  return hipGetLastError();
}

// Arguments of the per-tile sort (k_tile_sort, or the forward of a whole
// iteration, which sorts its tiles itself).
TileSortArgs tile_sort_args(const Plan& P, void* ws) {
  const bool splat = (P.cfg.flags & GS_SPLAT_BWD) != 0;
  TileSortArgs A{};
  A.cnt = ws_at<uint32_t>(ws, P.off_tile_cnt);
  A.tstart = ws_at<uint32_t>(ws, P.off_tile_start);
  A.fl = ws_at<int32_t>(ws, P.off_flags);
  const bool radix = (P.cfg.flags & GS_RADIX_BIN) != 0;  // (no scattered keys, no copies)
  A.skey = radix ? nullptr : ws_at<uint64_t>(ws, P.off_scatter);
  A.out = TileSortOut{ws_at<uint64_t>(ws, P.off_keys), ws_at<uint32_t>(ws, P.off_vals),
                      ws_at<uint32_t>(ws, P.off_sorted_rec),
                      radix ? nullptr : ws_at<uint32_t>(ws, P.off_pair_rec),
                      ws_at<Rec>(ws, P.off_rec), radix ? nullptr : ws_at<Rec>(ws, P.off_srec)};
  A.ranges = ws_at<uint32_t>(ws, P.off_ranges);
  A.fstart = splat ? ws_at<uint32_t>(ws, P.off_full_start) : nullptr;
  A.hstart = splat ? ws_at<uint32_t>(ws, P.off_half_start) : nullptr;
  A.bq = splat ? ws_at<uint2>(ws, P.off_bq) : nullptr;
  A.bq_stride = P.ckpt_slots;
  A.presorted = radix;
  A.long_after = !A.presorted;
  return A;
}

// defer_short_sorts: the lists of at most kTileSortSmall pairs are left to
// the forward (a whole iteration), which sorts each tile before compositing
// it; the long lists are sorted here in either case.
hipError_t launch_bin_sort(const Plan& P, void* ws, hipStream_t s, bool defer_short_sorts,
                           const StepAdvance* step, const Marks* marks) {
  const Marks none{};
  const Marks& mk = marks ? *marks : none;
  int32_t* fl = ws_at<int32_t>(ws, P.off_flags);
  uint32_t* tt = ws_at<uint32_t>(ws, P.off_tt);
  uint32_t* poff = ws_at<uint32_t>(ws, P.off_poff);
  uint32_t* tcnt = ws_at<uint32_t>(ws, P.off_tile_cnt);
  uint32_t* tstart = ws_at<uint32_t>(ws, P.off_tile_start);
  const bool splat = (P.cfg.flags & GS_SPLAT_BWD) != 0;
  const int T = P.vt.total_tiles;
  uint32_t* fstart = splat ? ws_at<uint32_t>(ws, P.off_full_start) : nullptr;
  uint32_t* hstart = splat ? ws_at<uint32_t>(ws, P.off_half_start) : nullptr;
  const uint2* chunk_cnt = ws_at<uint2>(ws, P.off_chunk_cnt);
  uint2* chunk_pre = ws_at<uint2>(ws, P.off_chunk_pre);
  uint4* long_list = ws_at<uint4>(ws, P.off_long);
  const bool radix = (P.cfg.flags & GS_RADIX_BIN) != 0;
  ScanArgs sa{chunk_cnt, chunk_pre, P.n_chunks, tcnt, tstart, (int64_t)T,
              splat ? ws_at<uint32_t>(ws, P.off_boff) : nullptr, fstart, hstart,
              ws_at<uint32_t>(ws, P.off_order), long_list, kScanBoth};
  // always launched, so that the flags are always set: one block for a
  // plan of one round, one block per round in three launches beyond
  const StepAdvance adv = step ? *step : StepAdvance{};
  auto scan = [&](const ScanArgs& a, const StepAdvance& st) {
    if (P.scan_rounds <= 1) {
      hipLaunchKernelGGL(k_scans, dim3(1), dim3(kScanBlock), 0, s, a, P.pair_cap, fl, st);
    } else {
      static_assert(sizeof(ScanPart) <= 64, "scan partial slot");
      ScanPart* part = ws_at<ScanPart>(ws, P.off_scan_part);
      const unsigned rounds = (unsigned)P.scan_rounds;
      hipLaunchKernelGGL(k_scan_reduce, dim3(rounds), dim3(kScanBlock), 0, s, a, part);
      hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, s, a, part, P.scan_rounds,
                         P.pair_cap, fl, st);
      hipLaunchKernelGGL(k_scan_down, dim3(rounds), dim3(kScanBlock), 0, s, a, part);
    }
  };
  if (radix) {
    ScanArgs sc = sa;
    sc.n_tiles = 0;
    sc.mode = kScanChunks;
    scan(sc, adv);
  } else {
    scan(sa, adv);
  }
  hipError_t e = mk.at(GS_MARK_BIN_SCAN, s);
  if (e != hipSuccess) return e;
  if (radix) {
    // records by depth, their pairs in that order, then the pairs by tile;
    // the list starts and ends found in the sorted keys give the per-tile
    // counts (the projection counted none), scanned like the projection's;
    // the per-tile pass (here, or the forward's when deferred) writes the
    // ranges and queue entries and zeroes the counters
    if ((e = launch_rb_generate(P, ws, s)) != hipSuccess) return e;
    if ((e = mk.at(GS_MARK_BIN_SCATTER, s)) != hipSuccess) return e;
    if ((e = launch_rb_tile_sort(P, ws, s)) != hipSuccess) return e;
    if ((e = mk.at(GS_MARK_BIN_SHORT_SORT, s)) != hipSuccess) return e;
    if ((e = launch_rb_runs(P, ws, s)) != hipSuccess) return e;
    ScanArgs st = sa;
    st.n_chunks = 0;
    st.mode = kScanTiles;
    scan(st, StepAdvance{});
    if (T > 0 && !defer_short_sorts) {
      hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)T), dim3(kWave), 0, s, tile_sort_args(P, ws));
    }
    if ((e = mk.at(GS_MARK_BIN_LONG_SORT, s)) != hipSuccess) return e;
    return hipGetLastError();
  }
  uint64_t* skey = ws_at<uint64_t>(ws, P.off_scatter);
  uint32_t* pair_rec = ws_at<uint32_t>(ws, P.off_pair_rec);
  if (P.n_chunks > 0) {
    const int64_t blocks = (P.n_chunks + 3) / 4;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, tt, poff, chunk_pre,
                       P.chunks_per_view, P.n_chunks, ws_at<ushort4>(ws, P.off_rect),
                       ws_at<Rec>(ws, P.off_rec), P.n, P.vt, fl, tstart, tcnt, skey, pair_rec,
                       ws_at<uint32_t>(ws, P.off_vis_list), ws_at<uint32_t>(ws, P.off_vis_clamp));
  }
  if ((e = mk.at(GS_MARK_BIN_SCATTER, s)) != hipSuccess) return e;
  if (T > 0) {
    // the per-tile pass (here, or the forward's when deferred) and the
    // long-list kernel each zero the counters they consume, so that every
    // counter is zero again after the binning of an iteration
    const TileSortArgs A = tile_sort_args(P, ws);
    if (!defer_short_sorts) hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)T), dim3(kWave), 0, s, A);
    if ((e = mk.at(GS_MARK_BIN_SHORT_SORT, s)) != hipSuccess) return e;
    // lists up to kTileSortMid pairs: a wavefront each; longer: a block each
    // (at most one long list per kTileSortSmall + 1 pairs of capacity; five
    // workgroups per CU are resident, the waves loop over the lists)
    const int64_t max_long = std::min<int64_t>(T, P.pair_cap / (kTileSortSmall + 1) + 1);
    const int mid_grid = (int)std::min<int64_t>((max_long + kMidWaves - 1) / kMidWaves, 1280);
    hipLaunchKernelGGL(k_tile_sort_mid, dim3((unsigned)mid_grid), dim3(kMidWaves * kWave), 0, s,
                       tcnt, fl, long_list, skey, A.out, defer_short_sorts ? 0 : 1);
    const int long_grid = (int)std::min<int64_t>(T, 512);  // two blocks per CU
    hipLaunchKernelGGL(k_tile_sort_long, dim3((unsigned)long_grid), dim3(kLongThreads), 0, s,
                       tcnt, fl, long_list, skey, A.out, defer_short_sorts ? 0 : 1);
  } else if ((e = mk.at(GS_MARK_BIN_SHORT_SORT, s)) != hipSuccess) {
    return e;
  }
  if ((e = mk.at(GS_MARK_BIN_LONG_SORT, s)) != hipSuccess) return e;
  return hipGetLastError();
}

// Rounds of the binning scan for a plan (a round = one block's share).
int64_t scan_rounds(const Plan& P) {
  const int64_t rt = ((int64_t)P.vt.total_tiles + kTileRound - 1) / kTileRound;
  const int64_t rc = (P.n_chunks + kChunkRound - 1) / kChunkRound;
  return std::max<int64_t>(1, std::max(rt, rc));
}

// Sorted pair values (generation indices) after launch_bin_sort.
uint32_t* sorted_vals(const Plan& P, void* ws) { return ws_at<uint32_t>(ws, P.off_vals); }

}  // namespace gs

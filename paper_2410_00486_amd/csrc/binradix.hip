// a2, second form (GS_RADIX_BIN): tile binning by two stable radix sorts,
// with no per-tile atomics and no per-tile sorts.
//
// The lists must be ordered by (tile, depth, generation index) (Sec.
// III-C-1: per-tile lists in depth order).  A record meets a tile at most
// once, and its pairs carry consecutive generation indices that grow with
// the record index, so the order within a tile is also (depth, record
// index).  Hence:
//   1. the visible records are listed in record order with their depth
//      bits as keys (positive floats: the bits order like the values) and
//      a 16-byte generation payload each (tile box, first generation
//      index, record id);
//   2. a stable LSD radix sort orders their list positions by depth (ties
//      keep record order); its last pass writes the records' payloads in
//      that order, so the generation reads them in sequence;
//   3. their pairs are generated in that order (a scan of the pair counts
//      gives each record its first slot), key = global tile id, values =
//      generation index and record id;
//   4. a stable LSD radix sort by tile id (only the bits the plan's tile
//      count needs) then leaves every tile's pairs contiguous, in depth
//      order, at exactly the list starts the binning scan computed; its
//      last pass writes the sorted outputs (keys, values and record ids)
//      directly.
// Every pass is an upsweep (per-block digit counts), a per-digit scan over
// the blocks and a downsweep that ranks a block's keys (stable: wave64
// ballots, in index order), reorders them in LDS and writes each digit's
// run contiguously.  Counts are read on the device (flags), grids are sized
// for the plan's capacities; graph-capturable, no spin-waits.
#include "tilesort.h"
#include "wavescan.h"

namespace gs {
namespace {

constexpr int kRbThreads = 256;
constexpr int kRbItems = 12;
constexpr int kRbTile = kRbThreads * kRbItems;  // keys per block
constexpr int kRbWaves = kRbThreads / kWave;
constexpr int kRbMaxBits = 9;  // tile passes: 18 bits of tile id in two
constexpr int kRbMaxRadix = 1 << kRbMaxBits;
// depth-sorted records per block of the pair generation (4 per thread)
constexpr int kGenRecs = 1024;
constexpr int kGenPer = kGenRecs / kRbThreads;

static_assert(kRbMaxRadix == 2 * kRbThreads, "two digits per thread in the block scans");

// Number of keys a pass sorts: a flag of the workspace, zero after a pair
// overflow (then nothing is generated or written).
__device__ __forceinline__ int64_t rb_count(const int32_t* fl, int which) {
  return fl[F_OVERFLOW] ? 0 : (int64_t)fl[which];
}

// Lanes of the wavefront whose digit equals this lane's (among `valid`
// lanes), from one ballot per digit bit.
__device__ __forceinline__ uint64_t rb_peers(uint32_t d, bool valid, int bits) {
  uint64_t peers = ballot64(valid);
  for (int b = 0; b < bits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = ballot64(bit);
    peers &= bit ? bb : ~bb;
  }
  return peers;
}

// Exclusive scan over the block's 256 threads of one value each; every
// thread of the block must call.  ws: kRbWaves words of LDS.
__device__ __forceinline__ uint32_t rb_block_exscan(uint32_t x, uint32_t* ws) {
  const int w = threadIdx.x / kWave, lane = lane_id();
  const uint32_t incl = scan_dpp<6>(x);
  if (lane == kWave - 1) ws[w] = incl;
  __syncthreads();
  uint32_t off = 0;
  for (int k = 0; k < w; ++k) off += ws[k];
  __syncthreads();  // ws is reused by the caller's next scan
  return off + incl - x;
}

// What the pair generation needs of a visible record, in one 16-byte word
// (one random read per record once the records are in depth order): its
// tile box (x0 | y0 << 16, x1 | y1 << 16), first generation index and
// record id.
__device__ __forceinline__ uint32_t pay_tiles(const uint4 p) {
  return ((p.y & 0xFFFFu) - (p.x & 0xFFFFu)) * ((p.y >> 16) - (p.x >> 16));
}

// 1. Visible records in record order: pair offset (first generation index),
// visible-list entry, depth key and generation payload.  One wavefront per
// chunk of 64 Gaussians of a view, at the positions the binning scan gave
// the chunk.
__global__ void __launch_bounds__(256) k_rb_visible(
    const uint32_t* __restrict__ tt, uint32_t* __restrict__ poff,
    const uint2* __restrict__ chunk_pre, int64_t chunks_per_view, int64_t n_chunks,
    const Rec* __restrict__ rec, const uint2* __restrict__ rect, int64_t n,
    const int32_t* __restrict__ fl, uint32_t* __restrict__ vis_list,
    uint32_t* __restrict__ vis_clamp, uint32_t* __restrict__ dkey, uint4* __restrict__ pay,
    uint32_t* __restrict__ zrec) {
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t gw = (int64_t)blockIdx.x * (256 / kWave) + w;  // chunk
  if (gw >= n_chunks) return;
  const int v = (int)(gw / chunks_per_view);
  const int64_t gi = (gw - (int64_t)v * chunks_per_view) * kWave + lane;
  const int64_t ri = (int64_t)v * n + gi;
  const bool over = fl[F_OVERFLOW] != 0;
  const uint32_t c = (gi < n && !over) ? tt[ri] : 0u;
  float z = 0.0f;
  uint32_t cbits = 0;
  if (c > 0) {
    z = rec[ri].z;
    cbits = rec[ri].clamp;  // (same line as the depth)
  }
  const uint32_t incl = scan_dpp<6>(c);
  const uint2 cp = chunk_pre[gw];
  const uint64_t vmask = ballot64(c > 0);
  if (c > 0) {
    const uint32_t p0 = cp.x + (incl - c);
    poff[ri] = p0;
    const uint32_t vp = cp.y + (uint32_t)__popcll(vmask & lanemask_lt());
    vis_list[vp] = (uint32_t)ri;
    vis_clamp[vp] = cbits;
    dkey[vp] = __float_as_uint(z);
    zrec[ri] = __float_as_uint(z);
    const uint2 b = rect[ri];
    pay[vp] = make_uint4(b.x, b.y, p0, (uint32_t)ri);
  }
}

// Upsweep: per-block counts of the digit (key >> shift) & (2^bits - 1),
// stored digit-major: hist[d * nb_cap + block].
__global__ void __launch_bounds__(kRbThreads) k_rb_hist(const uint32_t* __restrict__ keys,
                                                        const int32_t* __restrict__ fl, int which,
                                                        uint32_t* __restrict__ hist,
                                                        int64_t nb_cap, int shift, int bits) {
  const int64_t cnt = rb_count(fl, which);
  const int64_t base = (int64_t)blockIdx.x * kRbTile;
  if (base >= cnt) return;
  __shared__ uint32_t h[kRbWaves][kRbMaxRadix];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int k = threadIdx.x; k < kRbWaves * kRbMaxRadix; k += kRbThreads) (&h[0][0])[k] = 0u;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t lt = lanemask_lt();
#pragma unroll 4
  for (int r = 0; r < kRbItems; ++r) {
    const int64_t idx = base + (int64_t)w * (kWave * kRbItems) + r * kWave + lane;
    const bool valid = idx < cnt;
    const uint32_t d = valid ? (keys[idx] >> shift) & mask : 0u;
    const uint64_t peers = rb_peers(d, valid, bits);
    // one lane per distinct digit adds the digit's lanes (no two lanes of a
    // wavefront touch the same word; each wavefront has its own row)
    if (valid && (peers & lt) == 0) h[w][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  for (int d = threadIdx.x; d <= (int)mask; d += kRbThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kRbWaves; ++k) s += h[k][d];
    hist[(int64_t)d * nb_cap + blockIdx.x] = s;
  }
}

// One block per digit: exclusive scan of the digit's counts over the active
// blocks (in place); the digit's total to dtot.
__global__ void __launch_bounds__(kRbThreads) k_rb_digit_scan(uint32_t* __restrict__ hist,
                                                              const int32_t* __restrict__ fl,
                                                              int which,
                                                              uint32_t* __restrict__ dtot,
                                                              int64_t nb_cap) {
  const int64_t cnt = rb_count(fl, which);
  const int64_t nb = (cnt + kRbTile - 1) / kRbTile;
  uint32_t* row = hist + (int64_t)blockIdx.x * nb_cap;
  __shared__ uint32_t ws[kRbWaves];
  __shared__ uint32_t tot;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kRbThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t x = b < nb ? row[b] : 0u;
    const uint32_t ex = rb_block_exscan(x, ws);
    if (b < nb) row[b] = carry + ex;
    if (threadIdx.x == kRbThreads - 1) tot = ex + x;
    __syncthreads();
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Outputs of the last tile pass: the sorted lists.
struct RbEmit {
  uint64_t* keys;          // tile << 32 | depth bits
  uint32_t* vals;          // generation index
  uint32_t* sorted_rec;    // record id
  const uint32_t* zrec;    // depth bits by record id (gathered per pair)
  // the last depth pass instead (spay non-null): the generation payload of
  // each value's record in sorted order, no keys or values
  const uint4* pay;
  uint4* spay;
};

// Downsweep: stable ranking of the block's keys by digit, reorder in LDS,
// then each digit's run written contiguously at the digit's global offset
// (digit totals scanned over digits + the block's offset within the digit).
// EMIT: the last pass of the tile sort (keys are tile ids, values
// generation indices): writes the sorted lists instead of keys / values.
template <bool EMIT, bool TWO>
__global__ void __launch_bounds__(kRbThreads) k_rb_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const uint32_t* __restrict__ vals2_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, uint32_t* __restrict__ vals2_out, RbEmit E,
    const int32_t* __restrict__ fl, int which, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ dtot, int64_t nb_cap, int shift, int bits) {
  const int64_t cnt = rb_count(fl, which);
  const int64_t base = (int64_t)blockIdx.x * kRbTile;
  if (base >= cnt) return;
  __shared__ uint32_t wcnt[kRbWaves][kRbMaxRadix];
  __shared__ uint32_t lstart[kRbMaxRadix];
  __shared__ uint32_t gofs[kRbMaxRadix];
  __shared__ uint32_t ws[kRbWaves];
  // one staging buffer, reused for the keys, the values and the second
  // values in turn (a third of the LDS of staging all three, so more
  // workgroups per CU hide the memory latency)
  __shared__ uint32_t sbuf[kRbTile];
  const int w = threadIdx.x / kWave, lane = lane_id();
  // the two consecutive digits this thread handles in the block scans
  const int d0 = 2 * (int)threadIdx.x, d1 = d0 + 1;
  const uint32_t mask = (1u << bits) - 1u;
  const bool h0 = d0 <= (int)mask, h1 = d1 <= (int)mask;
  for (int k = threadIdx.x; k < kRbWaves * kRbMaxRadix; k += kRbThreads) (&wcnt[0][0])[k] = 0u;
  {
    const uint32_t x0 = h0 ? dtot[d0] : 0u, x1 = h1 ? dtot[d1] : 0u;
    const uint32_t ex = rb_block_exscan(x0 + x1, ws);  // (its barrier also orders the clear)
    if (h0) gofs[d0] = ex + hist[(int64_t)d0 * nb_cap + blockIdx.x];
    if (h1) gofs[d1] = ex + x0 + hist[(int64_t)d1 * nb_cap + blockIdx.x];
  }
  // (the values are loaded only when they are staged: fewer registers held
  // through the ranking)
  uint32_t key[kRbItems], rank[kRbItems];
  const uint64_t lt = lanemask_lt();
  const int64_t ibase = base + (int64_t)w * (kWave * kRbItems) + lane;
#pragma unroll
  for (int r = 0; r < kRbItems; ++r) {
    const int64_t idx = ibase + r * kWave;
    const bool valid = idx < cnt;
    key[r] = valid ? keys_in[idx] : 0u;
    const uint32_t d = (key[r] >> shift) & mask;
    const uint64_t peers = rb_peers(d, valid, bits);
    const uint64_t below = peers & lt;
    uint32_t old = 0;
    if (valid) old = wcnt[w][d];
    if (valid && below == 0) wcnt[w][d] = old + (uint32_t)__popcll(peers);
    rank[r] = valid ? old + (uint32_t)__popcll(below) : 0xFFFFFFFFu;
  }
  __syncthreads();
  {
    // per digit: exclusive prefix over the waves, then the block-local
    // start of the digit's run
    uint32_t t0 = 0, t1 = 0;
#pragma unroll
    for (int k = 0; k < kRbWaves; ++k) {
      if (h0) {
        const uint32_t c = wcnt[k][d0];
        wcnt[k][d0] = t0;
        t0 += c;
      }
      if (h1) {
        const uint32_t c = wcnt[k][d1];
        wcnt[k][d1] = t1;
        t1 += c;
      }
    }
    const uint32_t ex = rb_block_exscan(t0 + t1, ws);
    if (h0) lstart[d0] = ex;
    if (h1) lstart[d1] = ex + t0;
  }
  __syncthreads();
  // each item's slot in the block's digit order (kRbTile: none)
#pragma unroll
  for (int r = 0; r < kRbItems; ++r) {
    if (rank[r] != 0xFFFFFFFFu) {
      const uint32_t d = (key[r] >> shift) & mask;
      rank[r] = lstart[d] + wcnt[w][d] + rank[r];
    } else {
      rank[r] = kRbTile;
    }
  }
  const int nloc = (int)((cnt - base) < kRbTile ? (cnt - base) : kRbTile);
  // keys: staged, then each slot's global position (kept for the values)
  // and the key itself (kept by the last pass for its output keys)
#pragma unroll
  for (int r = 0; r < kRbItems; ++r)
    if (rank[r] < (uint32_t)kRbTile) sbuf[rank[r]] = key[r];
  __syncthreads();
  uint32_t opos[kRbItems], okey[kRbItems];
#pragma unroll
  for (int q = 0; q < kRbItems; ++q) {
    const int i = threadIdx.x + q * kRbThreads;
    okey[q] = i < nloc ? sbuf[i] : 0u;
    const uint32_t d = (okey[q] >> shift) & mask;
    opos[q] = i < nloc ? gofs[d] + (uint32_t)i - lstart[d] : 0u;
    if (!EMIT && keys_out && i < nloc) keys_out[opos[q]] = okey[q];
  }
  __syncthreads();
  // values
  {
    uint32_t val[kRbItems];
#pragma unroll
    for (int r = 0; r < kRbItems; ++r)
      val[r] = rank[r] < (uint32_t)kRbTile
                   ? (vals_in ? vals_in[ibase + r * kWave] : (uint32_t)(ibase + r * kWave))
                   : 0u;
#pragma unroll
    for (int r = 0; r < kRbItems; ++r)
      if (rank[r] < (uint32_t)kRbTile) sbuf[rank[r]] = val[r];
  }
  __syncthreads();
  if (!EMIT && E.spay) {
    // the records' payloads in depth order: gathered four per thread in
    // flight, stored in place of the values
    constexpr int G = 4;
#pragma unroll
    for (int q0 = 0; q0 < kRbItems; q0 += G) {
      uint4 pv[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int i = threadIdx.x + (q0 + u) * kRbThreads;
        pv[u] = i < nloc ? E.pay[sbuf[i]] : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int i = threadIdx.x + (q0 + u) * kRbThreads;
        if (i < nloc) E.spay[opos[q0 + u]] = pv[u];
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < kRbItems; ++q) {
      const int i = threadIdx.x + q * kRbThreads;
      if (i < nloc) {
        if constexpr (EMIT) E.vals[opos[q]] = sbuf[i];
        else vals_out[opos[q]] = sbuf[i];
      }
    }
  }
  if constexpr (TWO) {
    {
      uint32_t val2[kRbItems];
#pragma unroll
      for (int r = 0; r < kRbItems; ++r)
        val2[r] = rank[r] < (uint32_t)kRbTile ? vals2_in[ibase + r * kWave] : 0u;
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRbItems; ++r)
        if (rank[r] < (uint32_t)kRbTile) sbuf[rank[r]] = val2[r];
    }
    __syncthreads();
    if constexpr (!EMIT) {
#pragma unroll
      for (int q = 0; q < kRbItems; ++q) {
        const int i = threadIdx.x + q * kRbThreads;
        if (i < nloc) vals2_out[opos[q]] = sbuf[i];
      }
    } else {
      // the record ids came along as second values; each pair's key takes
      // the depth of its record (all of the thread's gathers in flight
      // before its stores)
      uint32_t rid[kRbItems], zb[kRbItems];
#pragma unroll
      for (int q = 0; q < kRbItems; ++q) {
        const int i = threadIdx.x + q * kRbThreads;
        rid[q] = i < nloc ? sbuf[i] : 0u;
        zb[q] = i < nloc ? E.zrec[rid[q]] : 0u;
      }
#pragma unroll
      for (int q = 0; q < kRbItems; ++q) {
        const int i = threadIdx.x + q * kRbThreads;
        if (i < nloc) {
          E.keys[opos[q]] = ((uint64_t)okey[q] << 32) | zb[q];
          E.sorted_rec[opos[q]] = rid[q];
        }
      }
    }
  } else {
    static_assert(TWO || !EMIT, "the last tile pass carries the record ids");
  }
}

// 3a. Pairs of each block of kGenRecs depth-sorted records.
__global__ void __launch_bounds__(kRbThreads) k_rb_gen_count(const uint4* __restrict__ spay,
                                                             const int32_t* __restrict__ fl,
                                                             uint32_t* __restrict__ part) {
  const int64_t V = rb_count(fl, F_VISIBLE);
  const int64_t base = (int64_t)blockIdx.x * kGenRecs;
  if (base >= V) return;
  __shared__ uint32_t ws[kRbWaves];
  uint32_t s = 0;
#pragma unroll
  for (int q = 0; q < kGenPer; ++q) {
    const int64_t j = base + q * kRbThreads + threadIdx.x;
    if (j < V) s += pay_tiles(spay[j]);
  }
  s = scan_dpp<6>(s);
  if (lane_id() == kWave - 1) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < kRbWaves; ++k) t += ws[k];
    part[blockIdx.x] = t;
  }
}

// 3b. One block: exclusive scan of the block pair counts (in place).
__global__ void __launch_bounds__(kRbThreads) k_rb_gen_scan(const int32_t* __restrict__ fl,
                                                            uint32_t* __restrict__ part) {
  const int64_t V = rb_count(fl, F_VISIBLE);
  const int64_t nb = (V + kGenRecs - 1) / kGenRecs;
  __shared__ uint32_t ws[kRbWaves];
  __shared__ uint32_t tot;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kRbThreads) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t x = b < nb ? part[b] : 0u;
    const uint32_t ex = rb_block_exscan(x, ws);
    if (b < nb) part[b] = carry + ex;
    if (threadIdx.x == kRbThreads - 1) tot = ex + x;
    __syncthreads();
    carry += tot;
    __syncthreads();
  }
}

// 3c. Pair generation in depth order: the block's records (4 consecutive
// per thread) get their first slots from a block scan plus the block's
// offset; the block's pairs are then spread evenly over the threads (each
// finds its record by binary search of the slots in LDS), so one large
// footprint does not serialise on one thread.  Writes the tile key, the
// generation index and the record id of every pair.
__global__ void __launch_bounds__(kRbThreads) k_rb_generate(
    const uint4* __restrict__ spay, int64_t n, ViewTable vt,
    const int32_t* __restrict__ fl, const uint32_t* __restrict__ part,
    uint32_t* __restrict__ tkey, uint32_t* __restrict__ gidx, uint32_t* __restrict__ ridx) {
  const int64_t V = rb_count(fl, F_VISIBLE);
  const int64_t base = (int64_t)blockIdx.x * kGenRecs;
  if (base >= V) return;
  __shared__ uint32_t s_pre[kGenRecs], s_p0[kGenRecs], s_t0[kGenRecs], s_rid[kGenRecs];
  __shared__ uint32_t s_bw[kGenRecs], s_tx[kGenRecs];
  __shared__ uint32_t ws[kRbWaves];
  __shared__ uint32_t s_total;
  uint32_t c[kGenPer], sum = 0;
#pragma unroll
  for (int q = 0; q < kGenPer; ++q) {
    const int64_t j = base + (int64_t)threadIdx.x * kGenPer + q;
    const int l = threadIdx.x * kGenPer + q;
    c[q] = 0u;
    if (j < V) {
      const uint4 p = spay[j];
      const uint32_t r = p.w;
      const int v = (int)(r / (uint64_t)n);
      const ViewInfo& vi = vt.v[v];
      c[q] = pay_tiles(p);
      s_rid[l] = r;
      s_p0[l] = p.z;
      s_bw[l] = (p.y & 0xFFFFu) - (p.x & 0xFFFFu);
      s_tx[l] = (uint32_t)vi.tiles_x;
      s_t0[l] = (uint32_t)(vi.tile_off + (int)(p.x >> 16) * vi.tiles_x + (int)(p.x & 0xFFFFu));
    }
    sum += c[q];
  }
  uint32_t run = rb_block_exscan(sum, ws);
#pragma unroll
  for (int q = 0; q < kGenPer; ++q) {
    // records past the end keep the block total: never chosen below
    s_pre[threadIdx.x * kGenPer + q] = run;
    run += c[q];
  }
  if (threadIdx.x == kRbThreads - 1) s_total = run;
  __syncthreads();
  const uint32_t total = s_total;
  const uint32_t q0 = part[blockIdx.x];
  for (uint32_t q = threadIdx.x; q < total; q += kRbThreads) {
    // owner: the last record whose first slot is <= q (every record here
    // has at least one pair, so the slots strictly increase)
    int lo = 0, hi = kGenRecs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const uint32_t k = q - s_pre[lo];
    const uint32_t bw = s_bw[lo];
    const uint32_t row = k / bw;
    const uint32_t t = s_t0[lo] + row * s_tx[lo] + (k - row * bw);
    const uint32_t g = s_p0[lo] + k;
    tkey[q0 + q] = t;
    gidx[q0 + q] = g;
    ridx[q0 + q] = s_rid[lo];
  }
}

// 5. Per-tile list bounds from the sorted keys (tile << 32 | depth): the
// first position of each tile's run to tstart, one past its last to cnt.
// Tiles without pairs keep cnt = 0 (the per-tile pass zeroed it).
__global__ void __launch_bounds__(kRbThreads) k_rb_runs(const uint64_t* __restrict__ keys,
                                                        const int32_t* __restrict__ fl,
                                                        uint32_t* __restrict__ tstart,
                                                        uint32_t* __restrict__ tend) {
  const int64_t P = rb_count(fl, F_PAIRS);
  const int64_t q = (int64_t)blockIdx.x * kRbThreads + threadIdx.x;
  if (q >= P) return;
  const uint32_t t = (uint32_t)(keys[q] >> 32);
  if (q == 0 || (uint32_t)(keys[q - 1] >> 32) != t) tstart[t] = (uint32_t)q;
  if (q == P - 1 || (uint32_t)(keys[q + 1] >> 32) != t) tend[t] = (uint32_t)(q + 1);
}

}  // namespace

namespace {

struct RbBuffers {
  const int32_t* fl;
  uint32_t *tt, *poff, *vis, *dk[2], *rid[2], *tk[2], *gx[2], *rx[2], *hist, *dtot, *part;
  uint4 *pay, *spay;
  RbEmit emit;
};

RbBuffers rb_buffers(const Plan& P, void* ws) {
  RbBuffers B;
  B.fl = ws_at<int32_t>(ws, P.off_flags);
  B.tt = ws_at<uint32_t>(ws, P.off_tt);
  B.poff = ws_at<uint32_t>(ws, P.off_poff);
  B.vis = ws_at<uint32_t>(ws, P.off_vis_list);
  for (int k = 0; k < 2; ++k) {
    B.dk[k] = ws_at<uint32_t>(ws, P.off_rb_dkey[k]);
    B.rid[k] = ws_at<uint32_t>(ws, P.off_rb_rid[k]);
    B.tk[k] = ws_at<uint32_t>(ws, P.off_rb_tkey[k]);
    B.gx[k] = ws_at<uint32_t>(ws, P.off_rb_gidx[k]);
    B.rx[k] = ws_at<uint32_t>(ws, P.off_rb_ridx[k]);
  }
  B.hist = ws_at<uint32_t>(ws, P.off_rb_hist);
  B.dtot = ws_at<uint32_t>(ws, P.off_rb_dtot);
  B.part = ws_at<uint32_t>(ws, P.off_rb_part);
  B.pay = ws_at<uint4>(ws, P.off_rb_pay);
  B.spay = ws_at<uint4>(ws, P.off_rb_spay);
  B.emit = RbEmit{ws_at<uint64_t>(ws, P.off_keys), ws_at<uint32_t>(ws, P.off_vals),
                  ws_at<uint32_t>(ws, P.off_sorted_rec), ws_at<uint32_t>(ws, P.off_rb_zrec),
                  nullptr, nullptr};
  return B;
}

// One stable pass over the keys counted by flag `which`; vin null: each
// key's value is its own position; vin2 / vout2: a second value array
// carried along (null: none); spay (no emit): write the payloads of the
// values' records in sorted order instead of keys and values.
void rb_pass(const RbBuffers& B, hipStream_t s, const uint32_t* kin, const uint32_t* vin,
             const uint32_t* vin2, uint32_t* kout, uint32_t* vout, uint32_t* vout2, bool emit,
             int which, int64_t nb_cap, int shift, int bits, uint4* spay = nullptr) {
  const dim3 grid((unsigned)nb_cap), block(kRbThreads);
  hipLaunchKernelGGL(k_rb_hist, grid, block, 0, s, kin, B.fl, which, B.hist, nb_cap, shift, bits);
  hipLaunchKernelGGL(k_rb_digit_scan, dim3(1u << bits), block, 0, s, B.hist, B.fl, which, B.dtot,
                     nb_cap);
#define GS_RB_SCATTER(E, T, OUT)                                                                \
  hipLaunchKernelGGL((k_rb_scatter<E, T>), grid, block, 0, s, kin, vin, vin2, kout, vout, vout2, \
                     OUT, B.fl, which, B.hist, B.dtot, nb_cap, shift, bits)
  if (emit) {  // (the lists' record ids come along as second values)
    GS_RB_SCATTER(true, true, B.emit);
  } else {
    if (vin2) GS_RB_SCATTER(false, true, RbEmit{});
    else GS_RB_SCATTER(false, false, (RbEmit{nullptr, nullptr, nullptr, nullptr, B.pay, spay}));
  }
#undef GS_RB_SCATTER
}

}  // namespace

// Workspace blocks of the radix binning: (record blocks, pair blocks, gen
// blocks) for a plan's record and pair capacities.
int64_t rb_blocks(int64_t count) { return (count + kRbTile - 1) / kRbTile; }
int64_t rb_gen_blocks(int64_t records) { return (records + kGenRecs - 1) / kGenRecs; }
int rb_max_radix() { return kRbMaxRadix; }

// Steps 1-3 of the radix binning (after the binning scan, which kept the
// per-tile counters): visible records, their depth sort, pair generation.
hipError_t launch_rb_generate(const Plan& P, void* ws, hipStream_t s) {
  const RbBuffers B = rb_buffers(P, ws);
  if (P.n_chunks <= 0 || P.rb_rec_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rb_visible, dim3((unsigned)((P.n_chunks + 3) / 4)), dim3(256), 0, s, B.tt,
                     B.poff, ws_at<uint2>(ws, P.off_chunk_pre), P.chunks_per_view, P.n_chunks,
                     ws_at<Rec>(ws, P.off_rec), ws_at<uint2>(ws, P.off_rect), P.n, B.fl, B.vis,
                     ws_at<uint32_t>(ws, P.off_vis_clamp), B.dk[0], B.pay,
                     ws_at<uint32_t>(ws, P.off_rb_zrec));
  // depth bits in four 8-bit passes; values: visible-list positions (the
  // first pass takes each key's own position); the last pass writes the
  // records' generation payloads in depth order instead
  // (dk0, -) -> (dk1, rid1) -> (dk0, rid0) -> (dk1, rid1) -> spay
  for (int p = 0; p < 4; ++p) {
    const uint32_t* kin = B.dk[p & 1];
    const uint32_t* vin = p == 0 ? nullptr : B.rid[p & 1];
    const bool last = p == 3;
    rb_pass(B, s, kin, vin, nullptr, last ? nullptr : B.dk[(p + 1) & 1],
            last ? nullptr : B.rid[(p + 1) & 1], nullptr, false, F_VISIBLE, P.rb_rec_blocks,
            8 * p, 8, last ? B.spay : nullptr);
  }
  const int64_t gb = rb_gen_blocks(P.n_rec);
  hipLaunchKernelGGL(k_rb_gen_count, dim3((unsigned)gb), dim3(kRbThreads), 0, s, B.spay, B.fl,
                     B.part);
  hipLaunchKernelGGL(k_rb_gen_scan, dim3(1), dim3(kRbThreads), 0, s, B.fl, B.part);
  hipLaunchKernelGGL(k_rb_generate, dim3((unsigned)gb), dim3(kRbThreads), 0, s, B.spay, P.n,
                     P.vt, B.fl, B.part, B.tk[0], B.gx[0], B.rx[0]);
  return hipGetLastError();
}

// Step 4: the pairs by tile id, as many passes of at most 9 bits as the
// plan's tile bits need (equal widths); the last writes the sorted lists.
hipError_t launch_rb_tile_sort(const Plan& P, void* ws, hipStream_t s) {
  const RbBuffers B = rb_buffers(P, ws);
  if (P.rb_pair_blocks <= 0) return hipSuccess;
  const int tb = P.tile_bits;
  const int passes = (tb + kRbMaxBits - 1) / kRbMaxBits;
  const int width = (tb + passes - 1) / passes;
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * width;
    const int bits = std::min(width, tb - shift);
    const bool last = p == passes - 1;
    rb_pass(B, s, B.tk[cur], B.gx[cur], B.rx[cur], last ? nullptr : B.tk[cur ^ 1],
            last ? nullptr : B.gx[cur ^ 1], last ? nullptr : B.rx[cur ^ 1], last, F_PAIRS,
            P.rb_pair_blocks, shift, bits);
    cur ^= 1;
  }
  return hipGetLastError();
}

// Step 5: list bounds per tile from the sorted keys (for the tile scan).
hipError_t launch_rb_runs(const Plan& P, void* ws, hipStream_t s) {
  if (P.rb_pair_blocks <= 0) return hipSuccess;
  const int64_t blocks = P.rb_pair_blocks * (kRbTile / kRbThreads);
  hipLaunchKernelGGL(k_rb_runs, dim3((unsigned)blocks), dim3(kRbThreads), 0, s,
                     ws_at<uint64_t>(ws, P.off_keys), ws_at<int32_t>(ws, P.off_flags),
                     ws_at<uint32_t>(ws, P.off_tile_start), ws_at<uint32_t>(ws, P.off_tile_cnt));
  return hipGetLastError();
}

}  // namespace gs

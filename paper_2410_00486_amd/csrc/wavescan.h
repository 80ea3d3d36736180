// Wavefront scan helpers shared by the binning kernels.
#pragma once

#include "gs_internal.h"

namespace gs {

// Inclusive wavefront scans with DPP (full-rate VALU, no LDS traffic): row
// shifts by 1, 2, 4, 8 within each 16-lane row, then the last lane of row 0
// and 2 into rows 1 and 3 (row_bcast:15) and of row 1 into rows 2 and 3
// (row_bcast:31).  Lanes shifted in from outside a row add 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
  const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)x);
  const uint32_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <typename U, int STEP>
__device__ __forceinline__ U dpp_step(U x) {
  if constexpr (sizeof(U) == 8) {
    if constexpr (STEP == 0) return dpp_u64<0x111>(x);
    else if constexpr (STEP == 1) return dpp_u64<0x112>(x);
    else if constexpr (STEP == 2) return dpp_u64<0x114>(x);
    else if constexpr (STEP == 3) return dpp_u64<0x118>(x);
    else if constexpr (STEP == 4) return dpp_u64<0x142, 0xA>(x);
    else return dpp_u64<0x143, 0xC>(x);
  } else {
    if constexpr (STEP == 0) return dpp_u32<0x111>(x);
    else if constexpr (STEP == 1) return dpp_u32<0x112>(x);
    else if constexpr (STEP == 2) return dpp_u32<0x114>(x);
    else if constexpr (STEP == 3) return dpp_u32<0x118>(x);
    else if constexpr (STEP == 4) return dpp_u32<0x142, 0xA>(x);
    else return dpp_u32<0x143, 0xC>(x);
  }
}

// Inclusive scan over the first 16 lanes (STEPS = 4) or the whole
// wavefront (STEPS = 6).
template <int STEPS, typename U>
__device__ __forceinline__ U scan_dpp(U x) {
  x += dpp_step<U, 0>(x);
  x += dpp_step<U, 1>(x);
  x += dpp_step<U, 2>(x);
  x += dpp_step<U, 3>(x);
  if constexpr (STEPS > 4) {
    x += dpp_step<U, 4>(x);
    x += dpp_step<U, 5>(x);
  }
  return x;
}

}  // namespace gs

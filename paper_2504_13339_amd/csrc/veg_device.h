// Device-only helpers shared by the HIP kernel sources of libveg.
#pragma once

#include "veg_internal.h"

namespace veg {

// ---------------------------------------------------------------------------------------
// wave64 primitives (DPP)
// ---------------------------------------------------------------------------------------

// DPP controls (gfx9): row_shr:n = 0x110+n, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_shift(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes of a wave (lanes that are inactive contribute
// whatever they hold, so call with the whole wave active).  Row-level Hillis-Steele steps
// with row_shr 1,2,4,8, then row_bcast:15 and row_bcast:31 carry the row totals.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
  v += dpp_shift<0x111, 0xf>(v);
  v += dpp_shift<0x112, 0xf>(v);
  v += dpp_shift<0x114, 0xf>(v);
  v += dpp_shift<0x118, 0xf>(v);
  v += dpp_shift<0x142, 0xa>(v);
  v += dpp_shift<0x143, 0xc>(v);
  return v;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_shift_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Sum over the 64 lanes; the total is valid in lane 63.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += dpp_shift_f<0x111, 0xf>(v);
  v += dpp_shift_f<0x112, 0xf>(v);
  v += dpp_shift_f<0x114, 0xf>(v);
  v += dpp_shift_f<0x118, 0xf>(v);
  v += dpp_shift_f<0x142, 0xa>(v);
  v += dpp_shift_f<0x143, 0xc>(v);
  return v;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

}  // namespace veg

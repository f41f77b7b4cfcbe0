// Reductions across one 64-lane wavefront without LDS: DPP lane moves inside
// each row of 16 lanes, then row broadcasts across the four rows.
// Every lane must be active; every lane receives the same (bitwise) result.
#pragma once

#include <hip/hip_runtime.h>

namespace ctm {

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  int lo = (int)(unsigned)(u & 0xffffffffull), hi = (int)(unsigned)(u >> 32);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// DPP move into the rows ROWMASK selects; the other rows receive `old`.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_rows_f64(double old, double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned long long o = (unsigned long long)__double_as_longlong(old);
  int lo = __builtin_amdgcn_update_dpp((int)(unsigned)(o & 0xffffffffull), (int)(unsigned)(u & 0xffffffffull), CTRL,
                                       ROWMASK, 0xf, false);
  int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(u >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror and
// row_mirror reduce inside each row of 16; row_bcast:15 (into rows 1, 3) and
// row_bcast:31 (into rows 2, 3) then leave the total in lane 63.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  v += dpp_rows_f64<0x142, 0xA>(0.0, v);
  v += dpp_rows_f64<0x143, 0xC>(0.0, v);
  return readlane_f64(v, 63);
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x141>(v));
  v = fmax(v, dpp_f64<0x140>(v));
  v = fmax(v, dpp_rows_f64<0x142, 0xA>(v, v));
  v = fmax(v, dpp_rows_f64<0x143, 0xC>(v, v));
  return readlane_f64(v, 63);
}

}  // namespace ctm

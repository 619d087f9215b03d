// wave_ops.h -- wave-level helpers for the FP64 kernels of Steps 1-3: DPP
// moves of doubles inside a 16-lane row, row reductions, refined hardware
// reciprocals, and the round-robin ("circle") pairing schedule.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace damf {

// DPP move of a double.  Every CTRL used here (quad_perm, row_mirror,
// row_half_mirror) reads a lane of the same 16-lane row with all rows and
// banks enabled, so every lane is written and the old value is never used:
// mov_dpp, which leaves it undefined, saves zeroing the destination.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a row, result in every lane of the row.
__device__ __forceinline__ double row_sum16(double x) {
  x += dpp_d<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_d<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_d<0x141>(x);  // row_half_mirror
  x += dpp_d<0x140>(x);  // row_mirror
  return x;
}

__device__ __forceinline__ double row_max16(double x) {
  x = fmax(x, dpp_d<0xB1>(x));
  x = fmax(x, dpp_d<0x4E>(x));
  x = fmax(x, dpp_d<0x141>(x));
  x = fmax(x, dpp_d<0x140>(x));
  return x;
}

// 1 / sqrt(x) and 1 / x for normal positive x: the hardware estimates
// refined by two Newton steps each (quadratic convergence from the
// estimate's error to about one ulp).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}
// One Newton step each: about 2^-46 relative from the hardware estimates,
// for quantities that need no more.
__device__ __forceinline__ double rsqrt_nr1(double x) {
  double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ double rcp_nr1(double x) {
  double y = __builtin_amdgcn_rcp(x);
  return y * fma(-x, y, 2.0);
}
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

// Circle schedule over NP players (NP even) in NP / 2 pairs (top[i],
// bottom[i]): between steps tops move right and bottoms left (top 0 stays,
// top 1 takes bottom 0, the last bottom takes the last top), so NP - 1 steps
// pair every two players once and end in the starting arrangement.  At step 0
// top i holds player i and bottom i player NP / 2 + i.
template <int NP>
__device__ __forceinline__ int circ_id0(int q) {
  constexpr int M = NP / 2;
  return (q < M - 1) ? (q + 1) : (M + (NP - 2 - q));
}
// player held by top slot i / bottom slot i after s steps
template <int NP>
__device__ __forceinline__ int j16_top_id(int i, int s) {
  if (i == 0) return 0;
  int q = (i - 1 - s) % (NP - 1);
  if (q < 0) q += NP - 1;
  return circ_id0<NP>(q);
}
template <int NP>
__device__ __forceinline__ int j16_bot_id(int i, int s) {
  int q = (NP - 2 - i - s) % (NP - 1);
  if (q < 0) q += NP - 1;
  return circ_id0<NP>(q);
}

}  // namespace damf

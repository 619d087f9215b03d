// common.h -- small device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch_geom.h"

namespace damf {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// |x| for max reductions that must not skip a NaN (fmaxf drops NaN operands):
// NaN becomes +inf, so a non-finite residual shows up as an infinite maximum.
__device__ __forceinline__ float nan_to_inf(float a) { return (a == a) ? a : INFINITY; }

// Lower bound in a sorted int32 array (global or LDS).
template <typename T>
__device__ __forceinline__ int64_t lower_bound(const T *a, int64_t n, T x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ---- precision form: a basis element as a pair of BF16 numbers in one
// 32-bit word, hi = bf16(x) in the upper half and lo = bf16(x - hi) in the
// lower half (round to nearest even); x ~ hi + lo to about 2^-16 relative.
__host__ __device__ __forceinline__ uint32_t bf16_bits_rne(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__host__ __device__ __forceinline__ float bf16_value(uint32_t b) {
  const uint32_t u = b << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
__host__ __device__ __forceinline__ uint32_t split_encode(float x) {
  const uint32_t h = bf16_bits_rne(x);
  const uint32_t l = bf16_bits_rne(x - bf16_value(h));
  return (h << 16) | l;
}
__host__ __device__ __forceinline__ float split_decode(uint32_t w) {
  return bf16_value(w >> 16) + bf16_value(w & 0xffffu);
}

// Element i of a basis stored as FP32 or, with split, as a BF16 pair.
__device__ __forceinline__ float basis_ld(const float *M, int64_t i, bool split) {
  return split ? split_decode(__float_as_uint(M[i])) : M[i];
}
__device__ __forceinline__ void basis_st(float *M, int64_t i, float v, bool split) {
  M[i] = split ? __uint_as_float(split_encode(v)) : v;
}

}  // namespace damf

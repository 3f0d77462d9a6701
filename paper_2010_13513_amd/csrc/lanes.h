// Wavefront lane shifts shared by the k-marching kernels (kernels.hip,
// ukernels.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace hhg {
namespace gen {
// DPP wave_shr:1 / wave_shl:1: the value held by lane L - 1 (from_prev) or
// L + 1 (from_next); the end lanes receive 0.
template <int CTRL>
__device__ __forceinline__ int lane_shift(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __int_as_float(lane_shift<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = lane_shift<CTRL>((int)(unsigned)(b & 0xffffffffull));
  const int hi = lane_shift<CTRL>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename T>
__device__ __forceinline__ T from_prev(T v) {
  return lane_shift<0x138>(v);
}
template <typename T>
__device__ __forceinline__ T from_next(T v) {
  return lane_shift<0x130>(v);
}
}  // namespace gen
}  // namespace hhg

// Device helpers shared by the kernel sources (representation types, the
// trilinear weights and the fixed-point rounding of the deposit).
#pragma once
#include "pic_internal.h"

namespace pic {
namespace {

template <int R>
struct RealOf {
  using T = float;
};
template <>
struct RealOf<PIC_REPR_FP64> {
  using T = double;
};

struct __align__(16) F4 {
  float x, y, z, w;
};
struct __align__(16) D4 {
  double x, y, z, w;
};
template <class T>
struct Vec4Of;
template <>
struct Vec4Of<float> {
  using type = F4;
};
template <>
struct Vec4Of<double> {
  using type = D4;
};

template <int D>
struct AccOf;
template <>
struct AccOf<PIC_DEP_FIXED64> {
  using type = unsigned long long;
};
template <>
struct AccOf<PIC_DEP_ATOMIC_FP32> {
  using type = float;
};
template <>
struct AccOf<PIC_DEP_ATOMIC_FP64> {
  using type = double;
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float floorT(float a) { return __builtin_floorf(a); }
__device__ __forceinline__ double floorT(double a) { return __builtin_floor(a); }
__device__ __forceinline__ float rintT(float a) { return __builtin_rintf(a); }
__device__ __forceinline__ double rintT(double a) { return __builtin_rint(a); }
__device__ __forceinline__ bool finiteT(float a) { return __builtin_isfinite(a); }
__device__ __forceinline__ bool finiteT(double a) { return __builtin_isfinite(a); }
__device__ __forceinline__ float absT(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double absT(double a) { return __builtin_fabs(a); }
template <class T>
__device__ __forceinline__ T two32();
template <>
__device__ __forceinline__ float two32<float>() { return 4294967296.0f; }
template <>
__device__ __forceinline__ double two32<double>() { return 4294967296.0; }

__device__ __forceinline__ int32_t pack_cell(int i, int j, int k) {
  return i | (j << kCellBits) | (k << (2 * kCellBits));
}

// Trilinear weights, corner n = a + 2b + 4c at offset (a, b, c).
template <class T>
__device__ __forceinline__ void weights(const T f[3], T W[8]) {
  const T wx0 = T(1) - f[0], wx1 = f[0];
  const T wy0 = T(1) - f[1], wy1 = f[1];
  const T wz0 = T(1) - f[2], wz1 = f[2];
  const T p00 = wx0 * wy0, p10 = wx1 * wy0, p01 = wx0 * wy1, p11 = wx1 * wy1;
  W[0] = p00 * wz0;
  W[1] = p10 * wz0;
  W[2] = p01 * wz0;
  W[3] = p11 * wz0;
  W[4] = p00 * wz1;
  W[5] = p10 * wz1;
  W[6] = p01 * wz1;
  W[7] = p11 * wz1;
}

// Fixed-point contribution at scale 2^32, rounded half to even. cw * 2^32 is
// exact in T and rint gives the integer nearest to it, so the value equals
// llrint((double)cw * 2^32).
template <class T>
__device__ __forceinline__ long long fixq(T cw) {
  return (long long)rintT(cw * two32<T>());
}

}  // namespace
}  // namespace pic

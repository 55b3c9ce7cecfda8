// gwf_arith.hpp -- reciprocals and square roots from the hardware estimates
// with their own refinement steps (host and device; the host build uses the
// library operations), for the dependent chains of the kernels where a
// correctly rounded division or square root would cost several times more.
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>

namespace gwf {

// 1/x for finite x != 0: the hardware reciprocal refined by two Newton
// steps (each squares the relative error), within an ulp or so of the
// rounded quotient; the host build divides.
__host__ __device__ inline double recip(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

// 1/sqrt(x) for finite x > 0: the hardware estimate y (relative error up to
// about 2^-23) refined by one third-order step, y (1 + e/2 + 3 e^2/8) with
// e = 1 - x y^2 (the series of (1 - e)^-1/2; the first term left out, 5e^3/16,
// is below 2^-66); the host build divides.
__host__ __device__ inline double rsqrt_d(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
#else
  return 1.0 / sqrt(x);
#endif
}

// sqrt(x) in FP32 from the hardware square root (about an ulp); the host
// build calls sqrtf.
__host__ __device__ inline float sqrtf_hw(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}

// 1/x in FP32 from the hardware reciprocal (about an ulp); the host build divides.
__host__ __device__ inline float recipf(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

}  // namespace gwf

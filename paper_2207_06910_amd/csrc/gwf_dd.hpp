// gwf_dd.hpp -- double-double arithmetic (a value as an unevaluated sum
// hi + lo of two doubles, |lo| <= ulp(hi)/2, about 106 significant bits),
// built from the error-free transformations: TwoSum (Knuth), FastTwoSum
// (Dekker) and the product error fma(a, b, -a*b).  Used by the inversion's
// extended-precision Cholesky, the GPU counterpart of the paper's
// arbitrary-precision inversion.
//
// Contraction of a*b + c into fma is switched off in these functions: the
// algorithms rely on the roundings as written, and dd_mul keeps its two
// cross products separate so that dd_mul(a, b) and dd_mul(b, a) are equal
// bit for bit (the inversion kernel needs that symmetry).
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>

namespace gwf {

struct dd {
  double hi, lo;
};

__host__ __device__ inline dd dd_from(double a) { return dd{a, 0.0}; }

// a + b exactly as s + e
__host__ __device__ inline dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return dd{s, e};
}

// a + b exactly as s + e, given |a| >= |b| (or a == 0)
__host__ __device__ inline dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double e = b - (s - a);
  return dd{s, e};
}

// a * b exactly as p + e
__host__ __device__ inline dd two_prod(double a, double b) {
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}

__host__ __device__ inline dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = two_sum(a.hi, b.hi);
  const dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}

__host__ __device__ inline dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

__host__ __device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

__host__ __device__ inline dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
  dd p = two_prod(a.hi, b.hi);
  const double c1 = a.hi * b.lo, c2 = a.lo * b.hi;
  p.lo += c1 + c2;
  return fast_two_sum(p.hi, p.lo);
}

__host__ __device__ inline dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
  const double q1 = a.hi / b.hi;
  const dd r = dd_sub(a, dd_mul(b, dd_from(q1)));
  const double q2 = r.hi / b.hi;
  const dd r2 = dd_sub(r, dd_mul(b, dd_from(q2)));
  const double q3 = r2.hi / b.hi;
  const dd q = fast_two_sum(q1, q2);
  return dd_add(q, dd_from(q3));
}

// sqrt(a), a >= 0 (0 for a <= 0): one Newton step on the double root
__host__ __device__ inline dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
  if (!(a.hi > 0.0)) return dd{0.0, 0.0};
  const double s = sqrt(a.hi);
  const dd s2 = two_prod(s, s);
  const double r = ((a.hi - s2.hi) - s2.lo + a.lo) / (2.0 * s);
  return fast_two_sum(s, r);
}

}  // namespace gwf

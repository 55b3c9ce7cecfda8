// gwf_invert.hpp -- the pairing schedule and the plane rotation of the
// one-sided Jacobi that gives the condition number of a Fisher matrix
// (host and device, so that the host test build runs the same code).
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>

namespace gwf {

// A column pair counts as orthogonal once |x_p . x_q| <= kJacobiTol |x_p| |x_q|:
// 64 u, above the rounding level of the inner product of two columns of
// length <= 14 that a rotation has just made orthogonal.  A pair left at
// this level moves the singular values by a relative O(P kJacobiTol) ~ 1e-13.
constexpr double kJacobiTol = 0x1p-47;

// Partner of column j at step t (0 <= t < M-1) of a sweep over M (even)
// columns: column M-1 stays, the others turn round a circle, pairs
// (t+i, t-i) mod (M-1); over the M-1 steps every pair meets once.  Columns
// j >= M pair with themselves.
template <int M>
__host__ __device__ inline int jacobi_partner(int j, int t) {
  if (j >= M) return j;
  if (j == M - 1) return t;
  if (j == t) return M - 1;
  int q = 2 * t - j;
  if (q < 0) q += M - 1;
  else if (q >= M - 1) q -= M - 1;
  return q;
}

// Rotation of the column pair (x_p, x_q) with ap = |x_p|^2, aq = |x_q|^2,
// gam = x_p . x_q: x_p' = c x_p - s x_q, x_q' = s x_p + c x_q, with
// t = s/c the smaller root of t^2 + 2 zeta t - 1 = 0, zeta = (aq-ap)/(2 gam),
// makes x_p' . x_q' vanish.  Returns false (c = 1, s = 0) for a pair that is
// already orthogonal to kJacobiTol.
__host__ __device__ inline bool hestenes_rotation(double ap, double aq, double gam, double& c,
                                                  double& s) {
  c = 1.0;
  s = 0.0;
  if (!(fabs(gam) > kJacobiTol * sqrt(ap * aq))) return false;
  const double zeta = (aq - ap) / (2.0 * gam);
  const double tn = fabs(zeta) > 1e150 ? 0.5 / zeta
                                       : copysign(1.0, zeta) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
  c = 1.0 / sqrt(fma(tn, tn, 1.0));
  s = c * tn;
  return true;
}

}  // namespace gwf

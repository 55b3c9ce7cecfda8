// gwf_invert.hpp -- the pairing schedule and the plane rotation of the
// one-sided Jacobi that gives the condition number of a Fisher matrix
// (host and device, so that the host test build runs the same code).
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>

#include "gwf_arith.hpp"

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

// Rotation of the column pair (x_p, x_q) with ap = |x_p|^2, aq = |x_q|^2 and
// gam = x_p . x_q: x_p' = c x_p - s x_q, x_q' = s x_p + c x_q makes
// x_p' . x_q' vanish when t = s/c is the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (aq - ap) / (2 gam), i.e. with d = aq - ap
// and r = sqrt(d^2 + 4 gam^2),
//   t = sign(d) 2 gam / (|d| + r),   c^2 = (1 + |d|/r) / 2,
// and then |x_p'|^2 = ap - t gam, |x_q'|^2 = aq + t gam.
// (d, 2 gam) are scaled by a power of two first (exact), so that
// rho = d^2 + 4 gam^2 lies in [1/4, 2); then 1/r from the refined reciprocal
// square root, u = |d| + r, t from the refined reciprocal of u, and
// c = sqrt(h) = h / sqrt(h) with h = u / (2 r) in [1/2, 1]: each within a
// few ulps, with no division and no library square root on the dependent
// chain of the sweep.  c comes from its own square root rather than from
// 1/sqrt(1 + t^2), one step shorter; c^2 (1 + t^2) = 1 in exact arithmetic.
// Returns false (c = 1, s = t = 0) for a pair that is already orthogonal to
// kJacobiTol, tested as gam^2 <= kJacobiTol^2 ap aq (no square root).
__host__ __device__ inline bool hestenes_rotation(double ap, double aq, double gam, double& c, double& s,
                                                  double& t) {
  c = 1.0;
  s = 0.0;
  t = 0.0;
  if (!(gam * gam > (kJacobiTol * kJacobiTol) * (ap * aq))) return false;
  const double dl = aq - ap, g2 = 2.0 * gam;
  int ex;
  frexp(fmax(fabs(dl), fabs(g2)), &ex);
  const double ds = ldexp(dl, -ex), gs = ldexp(g2, -ex);
  const double ad = fabs(ds);
  const double rho = fma(ds, ds, gs * gs);
  const double ri = rsqrt_d(rho);              // 1/r
  const double u = fma(rho, ri, ad);           // |d| + r
  t = (copysign(1.0, dl) * gs) * recip(u);
  const double h = 0.5 * (u * ri);
  c = h * rsqrt_d(h);
  s = c * t;
  return true;
}

// x . y in four interleaved partial sums added in a fixed order (short
// dependency chains); x . y and y . x are bitwise equal.
template <int P>
__host__ __device__ inline double col_dot(const double* x, const double* y) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
  for (int i = 0; i < P; i += 4) {
    s0 = fma(x[i], y[i], s0);
    if (i + 1 < P) s1 = fma(x[i + 1], y[i + 1], s1);
    if (i + 2 < P) s2 = fma(x[i + 2], y[i + 2], s2);
    if (i + 3 < P) s3 = fma(x[i + 3], y[i + 3], s3);
  }
  return (s0 + s1) + (s2 + s3);
}

// One column's part of a Jacobi step: x is column j, y its partner column q
// (q == j: no partner), nx and ny their squared norms as their owners hold
// them.  Both columns of a pair compute the same rotation from the same
// bits; the new column is c x + sg y, gam = x . y and tn = t of the rotation.
// Returns true if the pair was rotated (c = 1, sg = gam = tn = 0 otherwise).
template <int P>
__host__ __device__ inline bool jacobi_pair(const double* x, const double* y, double nx, double ny, int j,
                                            int q, double& c, double& sg, double& gam, double& tn) {
  c = 1.0;
  sg = 0.0;
  gam = 0.0;
  tn = 0.0;
  if (q == j) return false;
  gam = col_dot<P>(x, y);
  const bool first = j < q;
  double s;
  const bool rot = hestenes_rotation(first ? nx : ny, first ? ny : nx, gam, c, s, tn);
  sg = first ? -s : s;
  return rot;
}

// Column j's squared norm after the rotation of jacobi_pair (x already
// rotated): ap - t gam for the lower-index column, aq + t gam for the other,
// or the exact inner product where the update would have lost more than half
// of the norm to cancellation.
template <int P>
__host__ __device__ inline double rotated_norm(const double* x, double nx, double gam, double tn, bool first) {
  const double u = first ? fma(-tn, gam, nx) : fma(tn, gam, nx);
  return u >= 0.5 * nx ? u : col_dot<P>(x, x);
}

// The step applied to column j itself; nx is updated to its new squared norm.
template <int P>
__host__ __device__ inline bool jacobi_update(double* x, const double* y, double& nx, double ny, int j, int q) {
  double c, sg, gam, tn;
  const bool rot = jacobi_pair<P>(x, y, nx, ny, j, q, c, sg, gam, tn);
#pragma unroll
  for (int i = 0; i < P; ++i) x[i] = fma(sg, y[i], c * x[i]);
  if (rot) nx = rotated_norm<P>(x, nx, gam, tn, j < q);
  return rot;
}

}  // namespace gwf

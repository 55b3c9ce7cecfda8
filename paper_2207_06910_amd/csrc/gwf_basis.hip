// gwf_basis.hip -- the Fisher matrix in other parameter bases: chi_s, chi_a
// in place of chi1z, chi2z and Lambda~, delta Lambda~ in place of Lambda1,
// Lambda2 (the paper's combinations, sec. 2.1), and the component masses
// m1, m2 in place of (Mc, eta) (sec. 3.2).
//
// A Fisher matrix transforms as Gamma' = J^T Gamma J, J_ia = d native_i /
// d new_a at the event.  J differs from the identity only in a few columns:
//   chi_s, chi_a:  chi1 = chi_s + chi_a, chi2 = chi_s - chi_a;
//   Lambda~, dL~:  (Lambda1, Lambda2) = R A(eta)^-1 (Lambda~, dL~) with
//                  A = [[a, b], [c, d]] the paper's coefficients of
//                  S = Lambda1 + Lambda2 and D = Lambda1 - Lambda2 and
//                  R = [[1, 1], [1, -1]] / 2; at fixed (Lambda~, dL~) the
//                  Lambdas move with eta: g = d(Lambda1, Lambda2)/d eta
//                  = -R A^-1 A'(eta) (S, D);
//   m1, m2:        Mc = (m1 m2)^(3/5) M^(-1/5), eta = m1 m2 / M^2, M = m1 + m2,
//                  and eta (with the Lambdas that follow it) moves with m1, m2.
// So Gamma J is a few combinations of Gamma's columns, and J^T (Gamma J) the
// same combinations of its rows: one thread per event applies them to each
// row, then to each column, reading and writing the [P][P][n] arrays with
// consecutive events in consecutive lanes (in place if out == fisher).
#include "gwf_kernels.hpp"

namespace gwf {

namespace {

constexpr int kBBlock = 256;

struct BasisJ {
  bool chi, lam, m12;
  double dMc1, dMc2, de1, de2;   // d Mc / d m1,2 and d eta / d m1,2
  double K[2][2];                // d (Lambda1, Lambda2) / d (Lambda~, dL~)
  double g[2];                   // d (Lambda1, Lambda2) / d eta at fixed (Lambda~, dL~)
};

// x[P] (a row or a column) -> the same entries combined by J.
template <int P>
__device__ inline void apply_j(const BasisJ& b, double* x) {
  const double x0 = x[0], x1 = x[1];
  double xe = x1;
  if (P >= 13 && b.lam) {                 // P = 14: e0 (row 13) is not mixed
    const double x11 = x[11], x12 = x[12];
    xe = fma(x11, b.g[0], fma(x12, b.g[1], x1));
    x[11] = fma(x11, b.K[0][0], x12 * b.K[1][0]);
    x[12] = fma(x11, b.K[0][1], x12 * b.K[1][1]);
  }
  if (b.m12) {
    x[0] = fma(x0, b.dMc1, xe * b.de1);
    x[1] = fma(x0, b.dMc2, xe * b.de2);
  } else {
    x[1] = xe;
  }
  if (b.chi) {
    const double x9 = x[9], x10 = x[10];
    x[9] = x9 + x10;
    x[10] = x9 - x10;
  }
}

template <int P>
__global__ __launch_bounds__(kBBlock) void basis_kernel(BasisArgs a) {
  const int64_t e = (int64_t)blockIdx.x * kBBlock + threadIdx.x;
  if (e >= a.n) return;
  BasisJ b;
  b.chi = a.basis & 1u;
  b.lam = (a.basis & 2u) != 0;
  b.m12 = (a.basis & 4u) != 0;
  const double Mc = a.par[e], eta = a.par[a.ld + e];
  const double de = sqrt(fmax(1.0 - 4.0 * eta, 0.0));
  b.dMc1 = b.dMc2 = b.de1 = b.de2 = 0.0;
  if (b.m12) {
    const double M = Mc * pow(eta, -0.6);
    const double m1 = 0.5 * M * (1.0 + de), m2 = 0.5 * M * (1.0 - de);
    const double iM = 1.0 / M, iM3 = iM * iM * iM;
    b.dMc1 = Mc * (0.6 / m1 - 0.2 * iM);
    b.dMc2 = Mc * (0.6 / m2 - 0.2 * iM);
    b.de1 = m2 * (m2 - m1) * iM3;
    b.de2 = m1 * (m1 - m2) * iM3;
  }
  b.K[0][0] = b.K[0][1] = b.K[1][0] = b.K[1][1] = 0.0;
  b.g[0] = b.g[1] = 0.0;
  if (P >= 13 && b.lam) {
    const double e2 = eta * eta;
    const double p = 1.0 + 9.0 * eta - 11.0 * e2, pd = 9.0 - 22.0 * eta;
    const double r = 1.0 - 13272.0 / 1319.0 * eta + 8944.0 / 1319.0 * e2;
    const double rd = -13272.0 / 1319.0 + 2.0 * 8944.0 / 1319.0 * eta;
    const double t = 1.0 - 15910.0 / 1319.0 * eta + 32850.0 / 1319.0 * e2 + 3380.0 / 1319.0 * e2 * eta;
    const double td = -15910.0 / 1319.0 + 2.0 * 32850.0 / 1319.0 * eta + 3.0 * 3380.0 / 1319.0 * e2;
    const double dd = -2.0 / de;                                  // d sqrt(1 - 4 eta) / d eta
    const double A00 = 8.0 / 13.0 * (1.0 + 7.0 * eta - 31.0 * e2), A01 = 8.0 / 13.0 * de * p;
    const double A10 = 0.5 * de * r, A11 = 0.5 * t;
    const double B00 = 8.0 / 13.0 * (7.0 - 62.0 * eta), B01 = 8.0 / 13.0 * (dd * p + de * pd);
    const double B10 = 0.5 * (dd * r + de * rd), B11 = 0.5 * td;
    const double idet = 1.0 / (A00 * A11 - A01 * A10);
    const double I00 = A11 * idet, I01 = -A01 * idet, I10 = -A10 * idet, I11 = A00 * idet;   // A^-1
    // K = R A^-1
    b.K[0][0] = 0.5 * (I00 + I10); b.K[0][1] = 0.5 * (I01 + I11);
    b.K[1][0] = 0.5 * (I00 - I10); b.K[1][1] = 0.5 * (I01 - I11);
    // g = -R A^-1 A' (S, D)
    const double l1 = a.par[11 * a.ld + e], l2 = a.par[12 * a.ld + e];
    const double S = l1 + l2, D = l1 - l2;
    const double u0 = fma(B00, S, B01 * D), u1 = fma(B10, S, B11 * D);
    const double v0 = fma(I00, u0, I01 * u1), v1 = fma(I10, u0, I11 * u1);
    b.g[0] = -0.5 * (v0 + v1);
    b.g[1] = -0.5 * (v0 - v1);
  }
  const int64_t n = a.n;
  bool fin = true;
  // Gamma J: combine the columns of every row
#pragma unroll 1
  for (int r = 0; r < P; ++r) {
    double x[P];
#pragma unroll
    for (int c = 0; c < P; ++c) x[c] = a.fisher[((int64_t)r * P + c) * n + e];
    apply_j<P>(b, x);
#pragma unroll
    for (int c = 0; c < P; ++c) a.out[((int64_t)r * P + c) * n + e] = x[c];
  }
  // J^T (Gamma J): combine the rows of every column
#pragma unroll 1
  for (int c = 0; c < P; ++c) {
    double x[P];
#pragma unroll
    for (int r = 0; r < P; ++r) x[r] = a.out[((int64_t)r * P + c) * n + e];
    apply_j<P>(b, x);
#pragma unroll
    for (int r = 0; r < P; ++r) {
      a.out[((int64_t)r * P + c) * n + e] = x[r];
      fin = fin && isfinite(x[r]);
    }
  }
  if (a.status && !fin) a.status[e] |= kEvNonFinite;
}

}  // namespace

hipError_t launch_basis(const BasisArgs& a, int P, hipStream_t stream) {
  const unsigned blocks = (unsigned)((a.n + kBBlock - 1) / kBBlock);
  // P = 12 and 14 carry e0 as their last row, which no basis mixes
  if (P == 13) hipLaunchKernelGGL((basis_kernel<13>), dim3(blocks), dim3(kBBlock), 0, stream, a);
  else if (P == 11) hipLaunchKernelGGL((basis_kernel<11>), dim3(blocks), dim3(kBBlock), 0, stream, a);
  else if (P == 14) hipLaunchKernelGGL((basis_kernel<14>), dim3(blocks), dim3(kBBlock), 0, stream, a);
  else if (P == 12) hipLaunchKernelGGL((basis_kernel<12>), dim3(blocks), dim3(kBBlock), 0, stream, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace gwf

// gwf_invert.hip -- batched FP64 inversion of Fisher matrices (sec. 4.1).
//
// One lane per event, matrices of compile-time size P.  Steps, in the
// paper's order: normalise rows/columns by sqrt(diag) (skipped when a
// diagonal entry is not > 0); condition number of the normalised matrix as
// the ratio of its extreme |eigenvalues| (cyclic Jacobi, which resolves the
// small eigenvalues of a unit-diagonal positive matrix to high relative
// accuracy); no inversion above cond_max; Cholesky G^ = L L^T, L^-1 in place,
// G^-1 = L^-T L^-1; undo the normalisation; sigma_i = sqrt(Cov_ii) and the
// inversion error max_ij |(Gamma Cov - 1)_ij|.
//
// The working matrix lives in registers (packed upper triangle, all
// indices compile-time constants after unrolling); a second packed copy per
// lane lives in LDS as [entry][lane], consecutive lanes on consecutive doubles.
#include "gwf_kernels.hpp"

namespace gwf {

namespace {

// 32 lanes per workgroup (a half-filled wavefront): one lane per event is
// latency-bound, so twice as many waves as with full wavefronts spread the
// events over more SIMDs (measured on 10^4 13x13 matrices: 32 lanes as
// fast as 64 or slightly faster, 16 and 128 about 12% slower).
constexpr int kInvBlock = 32;

template <int P>
struct Packed {
  static constexpr int N = P * (P + 1) / 2;
  __host__ __device__ static constexpr int idx(int i, int j) {
    return i <= j ? i * P - (i * (i - 1)) / 2 + (j - i) : j * P - (j * (j - 1)) / 2 + (i - j);
  }
};

template <int P>
__device__ inline void jacobi_eigenvalues(double* A, double* ev) {
  using S = Packed<P>;
  for (int sweep = 0; sweep < 40; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int p = 0; p < P - 1; ++p) {
#pragma unroll
      for (int q = p + 1; q < P; ++q) {
        const double apq = A[S::idx(p, q)];
        const double app = A[S::idx(p, p)], aqq = A[S::idx(q, q)];
        if (apq != 0.0 && fabs(apq) > 1e-300 &&
            fabs(apq) > 0x1p-60 * sqrt(fabs(app) * fabs(aqq))) {
          rotated = true;
          const double th = (aqq - app) / (2.0 * apq);
          const double t = fabs(th) > 1e150 ? 0.5 / th
                                            : copysign(1.0, th) / (fabs(th) + sqrt(fma(th, th, 1.0)));
          const double c = 1.0 / sqrt(fma(t, t, 1.0));
          const double s = t * c;
          A[S::idx(p, p)] = app - t * apq;
          A[S::idx(q, q)] = aqq + t * apq;
          A[S::idx(p, q)] = 0.0;
#pragma unroll
          for (int r = 0; r < P; ++r) {
            if (r == p || r == q) continue;
            const double arp = A[S::idx(r, p)], arq = A[S::idx(r, q)];
            A[S::idx(r, p)] = c * arp - s * arq;
            A[S::idx(r, q)] = s * arp + c * arq;
          }
        }
      }
    }
    if (!rotated) break;
  }
#pragma unroll
  for (int i = 0; i < P; ++i) ev[i] = A[S::idx(i, i)];
}

template <int P>
__global__ __launch_bounds__(kInvBlock) void invert_kernel(InvertArgs a) {
  using S = Packed<P>;
  constexpr int N = S::N;
  __shared__ double B[N][kInvBlock];
  const int lane = threadIdx.x;
  const int64_t e = (int64_t)blockIdx.x * kInvBlock + lane;
  if (e >= a.n) return;
  const double nan = __builtin_nan("");
  int32_t st = a.status[e];
  auto fail = [&](int32_t bits) {
    st |= bits;
    for (int i = 0; i < P; ++i) {
      a.sigma[(int64_t)i * a.n + e] = nan;
      if (a.cov)
        for (int j = 0; j < P; ++j) a.cov[((int64_t)i * P + j) * a.n + e] = nan;
    }
    if (a.inv_err) a.inv_err[e] = nan;
    if (a.logdet) a.logdet[e] = nan;
    a.status[e] = st;
  };
  if (st & (kEvInvalid | kEvSkipped)) {
    if (a.cond) a.cond[e] = nan;
    fail(0);
    return;
  }
  double A[N], d[P];
  bool finite = true, normalise = true;
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = i; j < P; ++j) {
      const double g = a.fisher[((int64_t)i * P + j) * a.n + e];
      A[S::idx(i, j)] = g;
      finite = finite && isfinite(g);
    }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const double g = A[S::idx(i, i)];
    normalise = normalise && (g > 0.0);
  }
#pragma unroll
  for (int i = 0; i < P; ++i) d[i] = normalise ? sqrt(A[S::idx(i, i)]) : 1.0;
  if (!finite) {
    if (a.cond) a.cond[e] = nan;
    fail(kEvNonFinite);
    return;
  }
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = i; j < P; ++j) {
      const double h = A[S::idx(i, j)] / (d[i] * d[j]);
      A[S::idx(i, j)] = h;
      B[S::idx(i, j)][lane] = h;
    }
  // condition number
  double ev[P];
  jacobi_eigenvalues<P>(A, ev);
  double emax = 0.0, emin = INFINITY;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    emax = fmax(emax, fabs(ev[i]));
    emin = fmin(emin, fabs(ev[i]));
  }
  const double cond = emin > 0.0 ? emax / emin : INFINITY;
  if (a.cond) a.cond[e] = cond;
  if (!(cond <= a.cond_max)) {
    fail(kEvIllCond);
    return;
  }
  // Cholesky of the normalised matrix (reloaded from the LDS copy), lower
  // factor stored at idx(i, j), i >= j
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = i; j < P; ++j) A[S::idx(i, j)] = B[S::idx(i, j)][lane];
  bool pd = true;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    double dj = A[S::idx(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) dj = fma(-A[S::idx(j, k)], A[S::idx(j, k)], dj);
    pd = pd && (dj > 0.0);
    const double ljj = sqrt(fmax(dj, 0.0));
    A[S::idx(j, j)] = ljj;
    const double inv = 1.0 / ljj;
#pragma unroll
    for (int i = j + 1; i < P; ++i) {
      double s = A[S::idx(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) s = fma(-A[S::idx(i, k)], A[S::idx(j, k)], s);
      A[S::idx(i, j)] = s * inv;
    }
  }
  if (!pd) {
    fail(kEvNotPD);
    return;
  }
  // ln det Gamma = sum_i ln Gamma_ii + ln det of the normalised matrix
  //             = 2 sum_i ln(d_i L_ii)
  if (a.logdet) {
    double ld = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) ld += log(d[i] * A[S::idx(i, i)]);
    a.logdet[e] = 2.0 * ld;
  }
  // L^-1 in place, row by row, columns ascending
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const double inv_ii = 1.0 / A[S::idx(i, i)];
#pragma unroll
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < i; ++k) s = fma(A[S::idx(i, k)], A[S::idx(k, j)], s);
      A[S::idx(i, j)] = -s * inv_ii;
    }
    A[S::idx(i, i)] = inv_ii;
  }
  // C = L^-T L^-1: C_ij = sum_{k >= max(i,j)} Li_ki Li_kj; then undo normalisation
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = i; j < P; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < P; ++k) s = fma(A[S::idx(k, i)], A[S::idx(k, j)], s);
      B[S::idx(i, j)][lane] = s / (d[i] * d[j]);
    }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    a.sigma[(int64_t)i * a.n + e] = sqrt(B[S::idx(i, i)][lane]);
    if (a.cov)
#pragma unroll
      for (int j = 0; j < P; ++j) a.cov[((int64_t)i * P + j) * a.n + e] = B[S::idx(i, j)][lane];
  }
  if (a.inv_err) {
    double err = 0.0;
    for (int i = 0; i < P; ++i) {
      double g[P];
#pragma unroll
      for (int k = 0; k < P; ++k) g[k] = a.fisher[((int64_t)i * P + k) * a.n + e];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        double s = (i == j) ? -1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) s = fma(g[k], B[S::idx(k, j)][lane], s);
        err = fmax(err, fabs(s));
      }
    }
    a.inv_err[e] = err;
  }
  a.status[e] = st;
}

template <int P>
hipError_t launch_p(const InvertArgs& a, hipStream_t stream) {
  const unsigned blocks = (unsigned)((a.n + kInvBlock - 1) / kInvBlock);
  hipLaunchKernelGGL((invert_kernel<P>), dim3(blocks), dim3(kInvBlock), 0, stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_invert(const InvertArgs& a, int P, hipStream_t stream) {
  switch (P) {
    case 1: return launch_p<1>(a, stream);
    case 2: return launch_p<2>(a, stream);
    case 3: return launch_p<3>(a, stream);
    case 4: return launch_p<4>(a, stream);
    case 5: return launch_p<5>(a, stream);
    case 6: return launch_p<6>(a, stream);
    case 7: return launch_p<7>(a, stream);
    case 8: return launch_p<8>(a, stream);
    case 9: return launch_p<9>(a, stream);
    case 10: return launch_p<10>(a, stream);
    case 11: return launch_p<11>(a, stream);
    case 12: return launch_p<12>(a, stream);
    case 13: return launch_p<13>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gwf

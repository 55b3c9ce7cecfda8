// gwf_invert.hip -- batched FP64 inversion of Fisher matrices (sec. 4.1).
//
// Steps, in the paper's order: normalise rows/columns by sqrt(diag) (skipped
// when a diagonal entry is not > 0); condition number of the normalised
// matrix as the ratio of its extreme |eigenvalues|; no inversion above
// cond_max; Cholesky G^ = L L^T, L^-1, G^-1 = L^-T L^-1; undo the
// normalisation; sigma_i = sqrt(Cov_ii), ln det Gamma and the inversion error
// max_ij |(Gamma Cov - 1)_ij|.
//
// Sixteen lanes per matrix, lane j holding column j in registers; a
// wavefront (one workgroup) works on four matrices.
//
// Condition number.  The |eigenvalues| of the symmetric normalised matrix
// are its singular values, found by one-sided (Hestenes) Jacobi: at each
// step the columns are paired by a round-robin schedule, each lane fetches
// its partner's column through cross-lane permutes, and both lanes of a pair
// compute the same rotation from bitwise identical inputs and update their
// own column, so one step makes P/2 rotations with no further exchange.  For
// a matrix with unit diagonal the singular values come out with relative
// errors of order kappa u (Demmel and Veselic, SIAM J. Matrix Anal. Appl. 13,
// 1992), the accuracy of a two-sided Jacobi on the same matrix.
//
// Inversion.  The Cholesky factorisation is right-looking over columns: at
// step k the pivot lane's column is broadcast and every later column updates
// itself; the updates keep the two copies of each off-diagonal element
// bitwise equal, so lane j reads L_jk from its own registers.  Lane j then
// forms column j of L^-1 by forward substitution against L (staged in LDS),
// and column j of the upper triangle of C = L^-T L^-1 from the staged
// columns of L^-1.  Every element is computed with the same operations in
// the same order as the textbook one-thread-per-matrix loops (left-looking
// Cholesky, row-wise L^-1, C_ij = sum_{k >= max(i,j)} Li_ki Li_kj), so the
// lane layout changes no result bit.
#include "gwf_dd.hpp"
#include "gwf_invert.hpp"
#include "gwf_kernels.hpp"

namespace gwf {

namespace {

constexpr int kGroup = 16;                 // lanes per matrix: one per column, P <= 14
constexpr int kInvBlock = 64;              // one wavefront
constexpr int kGroups = kInvBlock / kGroup;
constexpr int kMaxSweeps = 40;

// Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b mod 8).
// Renumbered so that each XCD takes one contiguous range of matrices, the
// 128-byte lines of the [P][P][N] arrays (16 events, four workgroups) are
// fetched into one XCD's L2 only.  A bijection on [0, nb) for any nb.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % 8, t = b / 8, q = nb / 8, r = nb % 8;
  return x * q + (x < r ? x : r) + t;
}

// Kept parameters that are in event e's parameter set (bit i: kept i).
template <int P>
__device__ inline uint32_t kept_rows(const InvertArgs& a, int64_t e) {
  if (!a.par_mask) return (1u << P) - 1u;
  const uint32_t m = a.par_mask[e];
  uint32_t k = 0;
#pragma unroll
  for (int i = 0; i < P; ++i) k |= ((m >> a.keep[i]) & 1u) << i;
  return k;
}

// Entry (r, c) of the matrix that is inverted: the stored entry of kept
// parameters r and c with the prior added on the diagonal; a parameter
// outside the event's set (its bit clear in am) stands in as a unit row and
// column, which leaves the inverse of the rest unchanged.
__device__ inline double gamma_rc(const InvertArgs& a, int64_t e, uint32_t am, int r, int c) {
  if (!rows_in(am, r, c)) return r == c ? 1.0 : 0.0;
  double v = a.fisher[((int64_t)a.keep[r] * a.p_full + a.keep[c]) * a.n + e];
  if (r == c) v += a.prior[r];
  return v;
}

// Row j of the matrix that is inverted.
template <int P>
__device__ inline void load_row(const InvertArgs& a, int64_t e, uint32_t am, int j, double* row) {
#pragma unroll
  for (int k = 0; k < P; ++k) row[k] = gamma_rc(a, e, am, j, k);
}

// Column j of the normalised matrix (the kept upper triangle with the prior
// on the diagonal, divided by d_i d_j), the same bits as the values the
// kernel starts from; zeros where valid is false.
template <int P>
__device__ inline void load_col(const InvertArgs& a, int64_t e, uint32_t am, int j, bool valid,
                                const double* d, double dj, double* h) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double v = 0.0;
    if (valid) {
      const int r = i <= j ? i : j, c = i <= j ? j : i;
      v = gamma_rc(a, e, am, r, c) / (d[i] * dj);
    }
    h[i] = v;
  }
}

// The condition number of the normalised matrix from the columns X of its
// one-sided Jacobi (the norms are its singular values), the ill-conditioned
// flag and whether the matrix is inverted by its Cholesky factor.
template <int P>
__device__ inline void condition_of(const double* x, bool own, bool go0, bool pd, double cond_max,
                                    double& cond, bool& ill, bool& ok) {
  double smax = 0.0, smin = INFINITY;
  if (own) smax = smin = sqrt(col_dot<P>(x, x));
#pragma unroll
  for (int off = kGroup / 2; off >= 1; off >>= 1) {
    smax = fmax(smax, __shfl_xor(smax, off, kGroup));
    smin = fmin(smin, __shfl_xor(smin, off, kGroup));
  }
  cond = smin > 0.0 ? smax / smin : INFINITY;
  ill = go0 && !(cond <= cond_max);
  ok = go0 && !ill && pd;
}

__device__ inline dd shfl_dd(dd v, int src) { return dd{__shfl(v.hi, src, kGroup), __shfl(v.lo, src, kGroup)}; }

// At least 3 waves per SIMD: left free, the compiler spends all 256 registers
// on load scheduling and a SIMD runs one wave of this latency-bound kernel.
template <int P>
__global__ __launch_bounds__(kInvBlock, 3) void invert_kernel(InvertArgs a) {
  constexpr int M = P + (P & 1);           // a zero column makes the count even
  constexpr int LD = P + 1;
  // Two buffers per matrix (11.6 KB per workgroup at P = 13, so that the
  // 2500 workgroups of 10^4 matrices are resident at once):
  //   Gs: Gamma as stored (row i at Gs[g][i]), then column i of L^-1 at
  //       Gs[g][i], then Gamma again for the residual;
  //   Ls: column k of L at Ls[g][k] (1/L_kk on the diagonal), then column j
  //       of Cov at Ls[g][j].
  __shared__ double Gs[kGroups][P][LD];
  __shared__ double Ls[kGroups][P][LD];
  const int lane = threadIdx.x;
  const int g = lane / kGroup, j = lane % kGroup;
  const int64_t e = a.base + xcd_block(blockIdx.x, gridDim.x) * kGroups + g;
  const bool live = e < a.n;
  const bool own = live && j < P;          // lane owns a column of a real matrix
  const double nan = __builtin_nan("");

  int32_t st = live ? a.status[e] : kEvSkipped;
  const bool use = live && !(st & (kEvInvalid | kEvSkipped));
  const uint32_t am = live ? kept_rows<P>(a, e) : 0u;

  // ---- Gamma (kept rows and columns, prior on the diagonal), row j per lane, into LDS
  if (use && j < P) load_row<P>(a, e, am, j, Gs[g][j]);
  __syncthreads();

  // column j of the upper triangle (h_i = Gamma_{min(i,j), max(i,j)}) and the diagonal
  double h[P], dg[P];
  bool fin = true;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    h[i] = 0.0;
    dg[i] = 1.0;
    if (use) {
      dg[i] = Gs[g][i][i];
      if (j < P) {
        h[i] = i <= j ? Gs[g][i][j] : Gs[g][j][i];
        fin = fin && isfinite(h[i]);
      }
    }
  }
  const uint64_t badm = __ballot(!fin);
  const bool nonfinite = ((badm >> (g * kGroup)) & 0xffffull) != 0;
  const bool go0 = use && !nonfinite;
  bool normalise = true;
#pragma unroll
  for (int i = 0; i < P; ++i) normalise = normalise && (dg[i] > 0.0);
  double d[P], dj = 1.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    d[i] = normalise ? sqrt(dg[i]) : 1.0;
    if (i == j) dj = d[i];
  }
#pragma unroll
  for (int i = 0; i < P; ++i) h[i] = go0 ? h[i] / (d[i] * dj) : 0.0;


  // ---- Cholesky, right-looking over columns
  double l[P];
#pragma unroll
  for (int i = 0; i < P; ++i) l[i] = h[i];
  bool pd = true;
  double ljj = 1.0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const double piv = __shfl(l[k], k, kGroup);   // updated Gamma^_kk
    pd = pd && (piv > 0.0);
    const double lkk = sqrt(fmax(piv, 0.0));
    const double inv = 1.0 / lkk;
    const double ljk = l[k] * inv;                // this column's L_jk (j > k)
#pragma unroll
    for (int i = k + 1; i < P; ++i) {
      const double lik = __shfl(l[i], k, kGroup) * inv;
      if (j > k) l[i] = fma(-lik, ljk, l[i]);
      else if (j == k) l[i] = lik;
    }
    if (j == k) {
      ljj = lkk;
      l[k] = inv;
    }
  }
  // ln det Gamma = 2 sum_i ln(d_i L_ii)
  double ld = own ? log(dj * ljj) : 0.0;
#pragma unroll
  for (int off = kGroup / 2; off >= 1; off >>= 1) ld += __shfl_xor(ld, off, kGroup);

  // ---- L^-1, column j by forward substitution
  if (j < P) {
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (i >= j) Ls[g][j][i] = l[i];
  }
  __syncthreads();
  double y[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) s = fma(Ls[g][k][i], y[k], s);   // y_k = 0 for k < j
    const double inv_ii = Ls[g][i][i];
    y[i] = i < j ? 0.0 : i == j ? inv_ii : -s * inv_ii;
  }
  if (j < P) {
#pragma unroll
    for (int k = 0; k < P; ++k) Gs[g][j][k] = y[k];
  }
  __syncthreads();

  // ---- C_ij for i <= j, undone normalisation, both triangles into LDS
  if (j < P) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = i; k < P; ++k) s = fma(Gs[g][i][k], y[k], s);   // zero terms for k < j
      if (i <= j) {
        const double cij = s / (d[i] * dj);
        Ls[g][j][i] = cij;
        Ls[g][i][j] = cij;
      }
    }
  }
  __syncthreads();

  // ---- condition number: one-sided Jacobi on the normalised columns
  // (reloaded: the same bits as h).  A wavefront that holds a matrix the SVD
  // below inverts, or whose eigen-decomposition is wanted, accumulates the
  // rotations V as well (H V = X), so that the SVD needs no second Jacobi; X
  // and the condition number come out the same either way.
  const bool want_eig = a.eigval != nullptr || a.eigvec != nullptr;
  const bool need_v =
      __any(go0 && (a.method == 2 || a.method == 3 || (a.method == 1 && !pd))) || want_eig;
  double x[P];
  load_col<P>(a, e, am, j, go0 && j < P, d, dj, x);
  double cond;
  bool ill, ok, svd_done = false;
  if (need_v) {
    double vs[P];
#pragma unroll
    for (int i = 0; i < P; ++i) vs[i] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
      bool rotated = false;
      double nx = col_dot<P>(x, x);
#pragma unroll 1
      for (int t = 0; t < M - 1; ++t) {
        const int q = jacobi_partner<M>(j, t);
        double y[P], yv[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
          y[i] = __shfl(x[i], q, kGroup);
          yv[i] = __shfl(vs[i], q, kGroup);
        }
        const double ny = __shfl(nx, q, kGroup);
        double c, sg, gam, tn;
        const bool rot = jacobi_pair<P>(x, y, nx, ny, j, q, c, sg, gam, tn);
#pragma unroll
        for (int i = 0; i < P; ++i) {
          x[i] = fma(sg, y[i], c * x[i]);
          vs[i] = fma(sg, yv[i], c * vs[i]);
        }
        if (rot) {
          nx = rotated_norm<P>(x, nx, gam, tn, j < q);
          rotated = true;
        }
      }
      if (!__any(rotated)) break;
    }
    condition_of<P>(x, own, go0, pd, a.cond_max, cond, ill, ok);

    // ---- SVD inversions and eigen-decomposition, on request, from the Jacobi
    // above with the rotations V accumulated: H V = X = U diag(s) with
    // orthonormal U and V; then H^-1 = V diag(w) U^T with w = 1/s (or the
    // paper's truncated or dropped small singular values), and eigenvalue
    // j = sign(u_j . v_j) s_j with eigenvector v_j.  Only wavefronts holding
    // such a matrix run it (need_v held for them).
    const bool svd_grp = go0 && !ill && (a.method == 2 || a.method == 3 || (a.method == 1 && !pd));
    if (__any(svd_grp) || want_eig) {
      // the normalisation again from the stored diagonal (the same bits as d;
      // recomputed so that d need not stay in registers through this block)
      double dn[P], dnj = 1.0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        dn[i] = (go0 && normalise) ? sqrt(gamma_rc(a, e, am, i, i)) : 1.0;
        if (i == j) dnj = dn[i];
      }
      const double sj = sqrt(col_dot<P>(x, x));
      double smx = own ? sj : 0.0;
#pragma unroll
      for (int off = kGroup / 2; off >= 1; off >>= 1) smx = fmax(smx, __shfl_xor(smx, off, kGroup));
      const double inv_s = sj > 0.0 ? 1.0 / sj : 0.0;
#pragma unroll
      for (int i = 0; i < P; ++i) x[i] *= inv_s;                    // u_j
      const double lam = col_dot<P>(x, vs) >= 0.0 ? sj : -sj;

      if (want_eig) {
        // ascending position of this eigenvalue; eigenvector signed so that
        // its largest-magnitude component (the first, on ties) is positive
        int rank = 0;
#pragma unroll
        for (int m = 0; m < P; ++m) {
          const double lm = __shfl(lam, m, kGroup);
          if (lm < lam || (lm == lam && m < j)) ++rank;
        }
        double bv = -1.0, bs = 1.0;
#pragma unroll
        for (int i = 0; i < P; ++i)
          if (fabs(vs[i]) > bv) { bv = fabs(vs[i]); bs = vs[i]; }
        const double fl = bs < 0.0 ? -1.0 : 1.0;
        if (live && j < P) {
          if (a.eigval) a.eigval[(int64_t)rank * a.n + e] = go0 ? lam : nan;
          if (a.eigvec)
#pragma unroll
            for (int i = 0; i < P; ++i) a.eigvec[((int64_t)i * P + rank) * a.n + e] = go0 ? fl * vs[i] : nan;
        }
      }

      // H^-1 = V diag(w) U^T: U and w into Gs (w in the padding column), V
      // into Ls, then column j of the upper triangle, both triangles into Ls
      const double thr = a.svals_thresh * smx;
      double w = inv_s;
      if (sj < thr) {
        if (a.method == 3) w = 0.0;
        else if (a.method == 2 && a.truncate) w = 1.0 / thr;
      }
      if (svd_grp && j < P) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
          Gs[g][j][i] = x[i];
          Ls[g][j][i] = vs[i];
        }
        Gs[g][j][P] = w;
      }
      __syncthreads();
      double cc[P];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        double t = 0.0;
        if (svd_grp && j < P)
#pragma unroll
          for (int m = 0; m < P; ++m) t = fma(Ls[g][m][i] * Gs[g][m][P], Gs[g][m][j], t);
        cc[i] = t;
      }
      __syncthreads();
      if (svd_grp && j < P) {
#pragma unroll
        for (int i = 0; i < P; ++i)
          if (i <= j) {
            const double cij = cc[i] / (dn[i] * dnj);
            Ls[g][j][i] = cij;
            Ls[g][i][j] = cij;
          }
      }
      __syncthreads();
      // ln det Gamma from the singular values where the Cholesky failed and all
      // eigenvalues are positive: lsv sums 2 ln d_j + ln s_j = ln det Gamma,
      // while ld holds half of it on every path (the output doubles it)
      double lsv = own ? fma(2.0, log(dnj), log(sj)) : 0.0;
#pragma unroll
      for (int off = kGroup / 2; off >= 1; off >>= 1) lsv += __shfl_xor(lsv, off, kGroup);
      const uint64_t negm = __ballot(own && !(lam > 0.0));
      const bool allpos = ((negm >> (g * kGroup)) & 0xffffull) == 0;
      if (svd_grp && !pd) ld = allpos ? 0.5 * lsv : nan;
      svd_done = svd_grp;
      ok = ok || svd_done;
    }
  } else {
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
      bool rotated = false;
      // squared column norms: exact at the start of each sweep, then carried
      // through the rotations
      double nx = col_dot<P>(x, x);
#pragma unroll 1
      for (int t = 0; t < M - 1; ++t) {
        const int q = jacobi_partner<M>(j, t);
        double y[P];
#pragma unroll
        for (int i = 0; i < P; ++i) y[i] = __shfl(x[i], q, kGroup);
        const double ny = __shfl(nx, q, kGroup);
        if (jacobi_update<P>(x, y, nx, ny, j, q)) rotated = true;
      }
      if (!__any(rotated)) break;
    }
    condition_of<P>(x, own, go0, pd, a.cond_max, cond, ill, ok);
  }
  // ---- double-double Cholesky (method 4): normalisation, factorisation,
  // L^-1 and C = L^-T L^-1 again in double-double arithmetic (~106 bits), so
  // the covariance of the FP64 matrix comes out to about kappa 2^-104 before
  // its rounding to FP64 -- what the paper obtains with mpmath.  Same lane
  // layout and operation order as the FP64 steps; L and L^-1 are staged in
  // LDS as (hi in Ls, lo in Gs).
  if (a.method == 4) {
    const bool ddg = go0 && !ill;
    dd dn[P], dnj = dd_from(1.0);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      dn[i] = dd_from(1.0);
      if (ddg && normalise) dn[i] = dd_sqrt(dd_from(gamma_rc(a, e, am, i, i)));
      if (i == j) dnj = dn[i];
    }
    dd lq[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      lq[i] = dd_from(0.0);
      if (ddg && j < P) {
        const int r = i <= j ? i : j, c = i <= j ? j : i;
        lq[i] = dd_div(dd_from(gamma_rc(a, e, am, r, c)), dd_mul(dn[i], dnj));
      }
    }
    bool pdd = true;
    dd lqjj = dd_from(1.0);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const dd piv = shfl_dd(lq[k], k);
      pdd = pdd && (piv.hi > 0.0);
      const dd lkk = dd_sqrt(piv);
      const dd inv = dd_div(dd_from(1.0), lkk);
      const dd ljk = dd_mul(lq[k], inv);
#pragma unroll
      for (int i = k + 1; i < P; ++i) {
        const dd lik = dd_mul(shfl_dd(lq[i], k), inv);
        if (j > k) lq[i] = dd_sub(lq[i], dd_mul(lik, ljk));
        else if (j == k) lq[i] = lik;
      }
      if (j == k) {
        lqjj = lkk;
        lq[k] = inv;
      }
    }
    if (ddg && j < P) {
#pragma unroll
      for (int i = 0; i < P; ++i)
        if (i >= j) {
          Ls[g][j][i] = lq[i].hi;
          Gs[g][j][i] = lq[i].lo;
        }
    }
    __syncthreads();
    dd yq[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      dd sacc = dd_from(0.0);
#pragma unroll
      for (int k = 0; k < i; ++k) sacc = dd_add(sacc, dd_mul(dd{Ls[g][k][i], Gs[g][k][i]}, yq[k]));
      const dd inv_ii = dd{Ls[g][i][i], Gs[g][i][i]};
      yq[i] = i < j ? dd_from(0.0) : i == j ? inv_ii : dd_neg(dd_mul(sacc, inv_ii));
    }
    __syncthreads();
    if (ddg && j < P) {
#pragma unroll
      for (int k = 0; k < P; ++k) {
        Ls[g][j][k] = yq[k].hi;
        Gs[g][j][k] = yq[k].lo;
      }
    }
    __syncthreads();
    double cc[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      dd sacc = dd_from(0.0);
      if (ddg && j < P && i <= j) {
#pragma unroll
        for (int k = i; k < P; ++k) sacc = dd_add(sacc, dd_mul(dd{Ls[g][i][k], Gs[g][i][k]}, yq[k]));
        sacc = dd_div(sacc, dd_mul(dn[i], dnj));
      }
      cc[i] = sacc.hi + sacc.lo;
    }
    __syncthreads();
    if (ddg && j < P) {
#pragma unroll
      for (int i = 0; i < P; ++i)
        if (i <= j) {
          Ls[g][j][i] = cc[i];
          Ls[g][i][j] = cc[i];
        }
    }
    __syncthreads();
    // ln det from the double-double factor
    double ldd = own ? 2.0 * (log(dnj.hi) + dnj.lo / dnj.hi + log(lqjj.hi) + lqjj.lo / lqjj.hi) : 0.0;
#pragma unroll
    for (int off = kGroup / 2; off >= 1; off >>= 1) ldd += __shfl_xor(ldd, off, kGroup);
    pd = pdd;
    ld = 0.5 * ldd;
    ok = ddg && pdd;
  }
  // Gamma again (L2-resident) for the residual
  if (a.inv_err && ok && j < P) load_row<P>(a, e, am, j, Gs[g][j]);
  __syncthreads();

  // ---- outputs
  double cv[P];
#pragma unroll
  for (int k = 0; k < P; ++k) cv[k] = Ls[g][j < P ? j : 0][k];   // column j of Cov
  double err = 0.0;
  if (a.inv_err && ok) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double s = (i == j) ? -1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < P; ++k) s = fma(Gs[g][i][k], cv[k], s);
      if (j < P) err = fmax(err, fabs(s));
    }
  }
#pragma unroll
  for (int off = kGroup / 2; off >= 1; off >>= 1) err = fmax(err, __shfl_xor(err, off, kGroup));

  if (!live) return;
  if (use) {
    if (nonfinite) st |= kEvNonFinite;
    else if (ill) st |= kEvIllCond;
    else if (!pd && !svd_done) st |= kEvNotPD;
    else if (!pd && a.method == 1) st |= kEvSvd;
  }
  // column j of the covariance at its output position (marginalised
  // parameters have none; parameters outside the event's set give zeros)
  const int oj = j < P ? a.out_pos[j] : -1;
  if (oj >= 0) {
    const int64_t no = a.n_out;
    const bool inj = (am >> j) & 1u;
    a.sigma[oj * a.n + e] = (ok && inj) ? sqrt(Ls[g][j][j]) : nan;
    if (a.cov)
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int ik = a.out_pos[k];
        if (ik >= 0) a.cov[(ik * no + oj) * a.n + e] = ok ? (rows_in(am, j, k) ? cv[k] : 0.0) : nan;
      }
  }
  if (j == 0) {
    if (a.sky) {
      // sky localisation region (sec. 4.1) from the theta-phi block
      double area = nan;
      if (ok && rows_in(am, a.i_theta, a.i_phi)) {
        const double ctt = Ls[g][a.i_theta][a.i_theta], cpp = Ls[g][a.i_phi][a.i_phi];
        const double ctp = Ls[g][a.i_phi][a.i_theta];
        const double det = fma(ctt, cpp, -(ctp * ctp));
        if (det >= 0.0) area = a.sky_fac * fabs(sin(a.theta[e])) * sqrt(det);
      }
      a.sky[e] = area;
    }
    if (a.cond) a.cond[e] = go0 ? cond : nan;
    if (a.inv_err) a.inv_err[e] = ok ? err : nan;
    if (a.logdet) a.logdet[e] = ok ? 2.0 * ld : nan;
    a.status[e] = st;
  }
}

template <int P>
hipError_t launch_p(const InvertArgs& a0, hipStream_t stream) {
  InvertArgs a = a0;
  if (a.p_full == 0) {           // the whole matrix, no manipulations
    a.p_full = P;
    a.n_out = P;
    for (int i = 0; i < kMaxPar; ++i) {
      a.keep[i] = (int8_t)(i < P ? i : 0);
      a.out_pos[i] = (int8_t)(i < P ? i : -1);
      a.prior[i] = 0.0;
    }
    a.i_theta = a.i_phi = -1;
    a.sky = nullptr;
  }
  return launch_slices(a, a.n, kGroups, kInvBlock, [&](const InvertArgs& s, dim3 grid, dim3 block) {
    hipLaunchKernelGGL((invert_kernel<P>), grid, block, 0, stream, s);
  });
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
    case 14: return launch_p<14>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gwf

"""TEST INFRASTRUCTURE ONLY -- Fisher inversion in arbitrary precision.

The paper inverts Fisher matrices with mpmath (sec. 4.1).  Steps, in the
paper's order:

1. normalise rows and columns by the square root of the diagonal, so the
   matrix has a unit diagonal (skipped if any diagonal entry is zero);
2. Cholesky-factorise the normalised matrix, G^ = L L^T, and invert it as
   L^-T L^-1 (the default 'cho' method);
3. undo the normalisation;

plus the diagnostics: the condition number (ratio of the largest to the
smallest absolute eigenvalue, here of the normalised matrix), the
threshold above which no inversion is attempted (default 1e50), and the
inversion error eps = max_ij |(Gamma Gamma^-1 - 1)_ij|.

Status bits: 2 = not positive definite (Cholesky failed; the paper would fall
back to an SVD, here the event is only flagged), 4 = condition number above
the threshold.  Flagged events get NaN covariances.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

ST_NOT_PD = 2
ST_ILL_COND = 4


def _one(F: np.ndarray, cond_max: float, dps: int):
    P = F.shape[0]
    with mp.workdps(dps):
        G = mp.matrix(P, P)
        for i in range(P):
            for j in range(P):
                G[i, j] = mp.mpf(float(F[i, j]))
        diag = [G[i, i] for i in range(P)]
        # the paper skips the normalisation when a diagonal entry is zero; a
        # negative one (not positive definite) is treated the same way
        normalise = all(d > 0 for d in diag)
        dn = [mp.sqrt(d) if normalise else mp.mpf(1) for d in diag]
        Gh = mp.matrix(P, P)
        for i in range(P):
            for j in range(P):
                Gh[i, j] = G[i, j] / (dn[i] * dn[j])
        ev = mp.eigsy(Gh, eigvals_only=True)
        absev = [abs(e) for e in ev]
        cond = max(absev) / min(absev) if min(absev) > 0 else mp.inf
        status = 0
        if cond > cond_max:
            return None, float(cond), ST_ILL_COND
        try:
            L = mp.cholesky(Gh)
        except ValueError:
            return None, float(cond), ST_NOT_PD
        Li = mp.inverse(L)
        Ch = Li.T * Li
        C = np.zeros((P, P))
        for i in range(P):
            for j in range(P):
                C[i, j] = float(Ch[i, j] / (dn[i] * dn[j]))
        return C, float(cond), status


def covariance(fisher: np.ndarray, cond_max: float = 1e50, dps: int = 50, idx=None):
    """Invert fisher[P][P][N] (events last).  Returns a dict with cov[P][P][n],
    sigma[P][n], cond[n], inv_err[n] and status[n] for the selected events
    (all events, or those in idx).  inv_err is eps evaluated exactly on the
    FP64 values of Gamma and of the returned covariance."""
    P, _, N = fisher.shape
    idx = np.arange(N) if idx is None else np.asarray(idx)
    n = len(idx)
    cov = np.full((P, P, n), np.nan)
    sigma = np.full((P, n), np.nan)
    cond = np.zeros(n)
    inv_err = np.full(n, np.nan)
    status = np.zeros(n, dtype=np.int32)
    for k, e in enumerate(idx):
        F = np.array(fisher[:, :, e], dtype=np.float64)
        C, c, st = _one(F, cond_max, dps)
        cond[k] = c
        status[k] = st
        if C is None:
            continue
        cov[:, :, k] = C
        sigma[:, k] = np.sqrt(np.diag(C))
        with mp.workdps(dps):
            Fm = mp.matrix(F.tolist())
            Cm = mp.matrix(C.tolist())
            R = Fm * Cm
            inv_err[k] = float(max(abs(R[i, j] - (1 if i == j else 0))
                                   for i in range(P) for j in range(P)))
    return {"cov": cov, "sigma": sigma, "cond": cond, "inv_err": inv_err, "status": status}

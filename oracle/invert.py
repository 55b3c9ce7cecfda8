"""TEST INFRASTRUCTURE ONLY -- Fisher inversion in arbitrary precision.

The paper inverts Fisher matrices with mpmath (sec. 4.1).  Steps, in the
paper's order:

1. normalise rows and columns by the square root of the diagonal, so the
   matrix has a unit diagonal (skipped if any diagonal entry is zero);
2. Cholesky-factorise the normalised matrix, G^ = L L^T, and invert it as
   L^-T L^-1 (the default 'cho' method);
3. undo the normalisation;

or, on request, the SVD inversions the paper offers ('svd' with optional
truncation of small singular values, 'svd_reg' leaving them out), and the
SVD in place of a failed Cholesky (the paper's default behaviour);

plus the diagnostics: the condition number (ratio of the largest to the
smallest absolute eigenvalue, here of the normalised matrix), the
threshold above which no inversion is attempted (default 1e50), and the
inversion error eps = max_ij |(Gamma Gamma^-1 - 1)_ij|.

Per-event parameter sets (par_mask, bit i for parameter i): an event's
Fisher matrix is that of its own parameters, so only that block is inverted
(or decomposed); the covariance of a parameter outside the set is 0 in its
row and column and its sigma NaN (the layout the GPU library returns).

Status bits: 2 = not positive definite (Cholesky failed; the paper would fall
back to an SVD, here the event is only flagged), 4 = condition number above
the threshold.  Flagged events get NaN covariances.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

ST_NOT_PD = 2
ST_ILL_COND = 4
ST_SVD = 32          # Cholesky failed, inverted by SVD instead


def _one(F: np.ndarray, cond_max: float, dps: int, method: str = "cho", truncate: bool = False,
         thresh: float = 1e-15):
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
        Ch = None
        if method in ("cho", "cho_svd"):
            try:
                L = mp.cholesky(Gh)
                Li = mp.inverse(L)
                Ch = Li.T * Li
            except ValueError:
                if method == "cho":
                    return None, float(cond), ST_NOT_PD
                status = ST_SVD       # the paper's default: an SVD instead
        if Ch is None:
            Ch = _svd_inverse(Gh, method == "svd_reg", truncate and method == "svd", thresh)
        C = np.zeros((P, P))
        for i in range(P):
            for j in range(P):
                C[i, j] = float(Ch[i, j] / (dn[i] * dn[j]))
        return C, float(cond), status


def _svd_inverse(Gh, drop: bool, truncate: bool, thresh: float):
    """Inverse of Gh = U diag(s) V from its SVD, V^T diag(1/s) U^T (sec. 4.1):
    with ``truncate`` every s below thresh * max(s) is raised to that value;
    with ``drop`` (svd_reg) those singular values are left out."""
    U, S, V = mp.svd_r(Gh)
    P = Gh.rows
    smax = max(S[i] for i in range(P))
    w = []
    for i in range(P):
        s = S[i]
        if s < thresh * smax:
            if drop:
                w.append(mp.mpf(0))
                continue
            if truncate:
                s = thresh * smax
        w.append(1 / s)
    return V.T * mp.diag(w) * U.T


def _in_set(par_mask, e: int, i: int) -> bool:
    return par_mask is None or bool((int(par_mask[e]) >> i) & 1)


def eigen(fisher: np.ndarray, dps: int = 50, par_mask=None):
    """Eigenvalues (ascending) and eigenvectors of each normalised Fisher
    matrix (rows and columns divided by sqrt(diag), as for the inversion and
    its condition number): eigval[P][N], eigvec[P][P][N] with column r the
    eigenvector of eigenvalue r, signed so that its largest-magnitude
    component is positive.  A parameter outside the event's set (par_mask)
    is represented by a unit row and column (eigenvalue 1, eigenvector e_i)."""
    P, _, N = fisher.shape
    val = np.zeros((P, N))
    vec = np.zeros((P, P, N))
    for e in range(N):
        with mp.workdps(dps):
            def entry(i, j):
                if _in_set(par_mask, e, i) and _in_set(par_mask, e, j):
                    return mp.mpf(float(fisher[i, j, e]))
                return mp.mpf(1) if i == j else mp.mpf(0)
            G = mp.matrix([[entry(i, j) for j in range(P)] for i in range(P)])
            normalise = all(G[i, i] > 0 for i in range(P))
            dn = [mp.sqrt(G[i, i]) if normalise else mp.mpf(1) for i in range(P)]
            for i in range(P):
                for j in range(P):
                    G[i, j] = G[i, j] / (dn[i] * dn[j])
            E, Q = mp.eigsy(G)
            for r in range(P):
                val[r, e] = float(E[r])
                col = [Q[i, r] for i in range(P)]
                big = max(range(P), key=lambda i: abs(col[i]))
                sgn = 1 if col[big] > 0 else -1
                for i in range(P):
                    vec[i, r, e] = float(sgn * col[i])
    return val, vec


def covariance(fisher: np.ndarray, cond_max: float = 1e50, dps: int = 50, idx=None, method: str = "cho",
               truncate: bool = False, svals_thresh: float = 1e-15, par_mask=None):
    """Invert fisher[P][P][N] (events last).  Returns a dict with cov[P][P][n],
    sigma[P][n], cond[n], inv_err[n] and status[n] for the selected events
    (all events, or those in idx).  inv_err is eps evaluated exactly on the
    FP64 values of Gamma and of the returned covariance.  method: "cho"
    (failed Cholesky flagged), "cho_svd" (the paper's default: an SVD where
    the Cholesky fails, status ST_SVD), "svd" (with ``truncate``: singular
    values below svals_thresh * max raised to it) or "svd_reg" (those left
    out).  par_mask [N] (or None): each event's parameter set; only that
    block is inverted."""
    P, _, N = fisher.shape
    idx = np.arange(N) if idx is None else np.asarray(idx)
    n = len(idx)
    cov = np.full((P, P, n), np.nan)
    sigma = np.full((P, n), np.nan)
    cond = np.zeros(n)
    inv_err = np.full(n, np.nan)
    status = np.zeros(n, dtype=np.int32)
    for k, e in enumerate(idx):
        sel = [i for i in range(P) if _in_set(par_mask, e, i)]
        if not sel:                      # an empty parameter set: nothing to invert
            cov[:, :, k], cond[k], inv_err[k] = 0.0, 1.0, 0.0
            continue
        F = np.array(fisher[np.ix_(sel, sel, [e])][:, :, 0], dtype=np.float64)
        C, c, st = _one(F, cond_max, dps, method, truncate, svals_thresh)
        cond[k] = c
        status[k] = st
        if C is None:
            continue
        cov[:, :, k] = 0.0
        cov[np.ix_(sel, sel, [k])] = C[:, :, None]
        sigma[sel, k] = np.sqrt(np.diag(C))
        with mp.workdps(dps):
            Fm = mp.matrix(F.tolist())
            Cm = mp.matrix(C.tolist())
            R = Fm * Cm
            inv_err[k] = float(max(abs(R[i, j] - (1 if i == j else 0))
                                   for i in range(len(sel)) for j in range(len(sel))))
    return {"cov": cov, "sigma": sigma, "cond": cond, "inv_err": inv_err, "status": status}


# ---------------------------------------------------------------------------
# Covariance epilogue (sec. 4.2 and the sky-localisation formula of sec. 4.1).
#
# Order, as the paper describes the manipulations: parameters held at their
# fiducial values are removed from the Fisher matrix before inversion; a
# diagonal Gaussian prior (its inverse variances) is added to the remaining
# matrix before inversion; the result is inverted as above; the sky area is
# taken from the covariance of the inverted matrix; parameters marginalised
# over are removed from the covariance after inversion.

def fix_params(fisher: np.ndarray, fixed) -> tuple[np.ndarray, np.ndarray]:
    """Remove the rows and columns of the parameters in ``fixed`` (indices
    into the P parameters) from fisher[P][P][N].  Returns the reduced matrix
    and the original indices of the parameters it keeps, in order."""
    P = fisher.shape[0]
    keep = np.array([i for i in range(P) if i not in set(int(f) for f in fixed)], dtype=np.int64)
    return fisher[np.ix_(keep, keep)], keep


def add_prior(fisher: np.ndarray, values, idx) -> np.ndarray:
    """Add values[k] to the diagonal entry idx[k] of every matrix (the
    inverse variance of a Gaussian prior on that parameter)."""
    out = np.array(fisher, dtype=np.float64, copy=True)
    for v, i in zip(values, idx):
        out[int(i), int(i)] += float(v)
    return out


def marginalise(cov: np.ndarray, over) -> tuple[np.ndarray, np.ndarray]:
    """Remove the rows and columns of the parameters in ``over`` from the
    covariance cov[P][P][N]; returns it and the indices kept."""
    return fix_params(cov, over)


def sky_area(cov: np.ndarray, theta: np.ndarray, i_theta: int, i_phi: int, perc_level: float = 90.0,
             units: str = "SqDeg", dps: int = 30) -> np.ndarray:
    """Sky localisation region containing perc_level percent of the
    probability,
        Delta Omega = -2 pi |sin theta| sqrt(C_tt C_pp - C_tp^2) ln(1 - X/100),
    in steradians or square degrees, from the covariance entries of the
    polar angle theta and the azimuth phi (NaN where the 2 x 2 determinant is
    negative or an entry is not finite)."""
    N = cov.shape[2]
    out = np.full(N, np.nan)
    with mp.workdps(dps):
        lnq = mp.log(1 - mp.mpf(perc_level) / 100)
        conv = (180 / mp.pi) ** 2 if units == "SqDeg" else mp.mpf(1)
        for e in range(N):
            ctt, cpp, ctp = cov[i_theta, i_theta, e], cov[i_phi, i_phi, e], cov[i_theta, i_phi, e]
            if not (np.isfinite(ctt) and np.isfinite(cpp) and np.isfinite(ctp)):
                continue
            det = mp.mpf(float(ctt)) * mp.mpf(float(cpp)) - mp.mpf(float(ctp)) ** 2
            if det < 0:
                continue
            out[e] = float(-2 * mp.pi * abs(mp.sin(mp.mpf(float(theta[e])))) * mp.sqrt(det) * lnq * conv)
    return out


def covariance_epilogue(fisher: np.ndarray, fixed=(), prior=None, marg=(), theta=None,
                        i_theta: int = 3, i_phi: int = 4, perc_level: float = 90.0, units: str = "SqDeg",
                        cond_max: float = 1e50, dps: int = 50, method: str = "cho", truncate: bool = False,
                        svals_thresh: float = 1e-15, par_mask=None):
    """The manipulations in order: fix -> prior -> invert -> sky area ->
    marginalise.  ``prior`` maps parameter index (of the full P) -> inverse
    prior variance.  ``i_theta``/``i_phi`` are indices of the full P; both must
    be kept for the sky area.  Returns the dictionary of ``covariance`` for
    the inverted matrix, plus ``cov_out``/``sigma_out`` after
    marginalisation, ``keep``/``out`` (original indices), ``sky`` and
    ``fisher_inverted`` (the matrix that was inverted).  par_mask [N] (bit i:
    parameter i of the full P, or None): each event's parameter set; the
    sky area is NaN for an event without theta or phi."""
    F, keep = fix_params(np.asarray(fisher, dtype=np.float64), fixed)
    pos = {int(k): i for i, k in enumerate(keep)}
    if prior:
        F = add_prior(F, list(prior.values()), [pos[int(i)] for i in prior.keys()])
    kmask = None
    if par_mask is not None:
        kmask = np.array([sum(((int(m) >> int(kk)) & 1) << i for i, kk in enumerate(keep)) for m in par_mask])
    res = covariance(F, cond_max=cond_max, dps=dps, method=method, truncate=truncate,
                     svals_thresh=svals_thresh, par_mask=kmask)
    res["fisher_inverted"] = F
    res["keep"] = keep
    if theta is not None:
        res["sky"] = sky_area(res["cov"], np.asarray(theta), pos[i_theta], pos[i_phi], perc_level, units)
        if kmask is not None:
            has = (((kmask >> pos[i_theta]) & 1) & ((kmask >> pos[i_phi]) & 1)).astype(bool)
            res["sky"][~has] = np.nan
    over = [pos[int(m)] for m in marg]
    cov_out, kept_pos = marginalise(res["cov"], over)
    res["cov_out"] = cov_out
    res["sigma_out"] = res["sigma"][kept_pos]
    res["out"] = keep[kept_pos]
    return res

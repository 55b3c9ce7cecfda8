"""TEST INFRASTRUCTURE ONLY -- the Fisher matrix in other parameter bases.

The native rows are (Mc, eta, dL, theta, phi, iota, psi, tc, Phic, chi1z,
chi2z[, Lambda1, Lambda2]).  The paper also computes the Fisher matrix in
terms of chi_s, chi_a (its eq. for the spin combinations), of the tidal
combinations Lambda~, delta Lambda~ (its eq. citing Wade et al.), and of the
component masses m1, m2 in place of (Mc, eta) (sec. 3.2, the use_m1m2 flag).
A Fisher matrix transforms as Gamma' = J^T Gamma J with J_ia = d(native i) /
d(new a) at the event; here J is obtained by differentiating the map from
the new parameters to the native ones numerically at 40 digits (mpmath), so
it shares no algebra with the GPU's closed-form Jacobian.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

CHI_SA = 1
LAMBDA_TILDE = 2
M1M2 = 4


def _tidal_coeffs(eta):
    """Lambda~ = a S + b D, delta Lambda~ = c S + d D, S = L1 + L2, D = L1 - L2."""
    de = mp.sqrt(1 - 4 * eta)
    a = mp.mpf(8) / 13 * (1 + 7 * eta - 31 * eta ** 2)
    b = mp.mpf(8) / 13 * de * (1 + 9 * eta - 11 * eta ** 2)
    c = mp.mpf(1) / 2 * de * (1 - mp.mpf(13272) / 1319 * eta + mp.mpf(8944) / 1319 * eta ** 2)
    d = mp.mpf(1) / 2 * (1 - mp.mpf(15910) / 1319 * eta + mp.mpf(32850) / 1319 * eta ** 2
                         + mp.mpf(3380) / 1319 * eta ** 3)
    return a, b, c, d


def new_parameters(par, basis):
    """The event's parameters in the new basis (mpf list), from native ones."""
    p = [mp.mpf(float(x)) for x in par]
    P = len(p)
    out = list(p)
    if basis & M1M2:
        Mc, eta = p[0], p[1]
        M = Mc * eta ** (mp.mpf(-3) / 5)
        de = mp.sqrt(1 - 4 * eta)
        out[0], out[1] = M * (1 + de) / 2, M * (1 - de) / 2
    if basis & CHI_SA:
        out[9], out[10] = (p[9] + p[10]) / 2, (p[9] - p[10]) / 2
    if basis & LAMBDA_TILDE and P >= 13:
        a, b, c, d = _tidal_coeffs(p[1])
        S, D = p[11] + p[12], p[11] - p[12]
        out[11], out[12] = a * S + b * D, c * S + d * D
    return out


def native_from_new(q, basis):
    """Inverse map: native parameters from new ones (mpf list)."""
    q = list(q)
    P = len(q)
    out = list(q)
    if basis & M1M2:
        m1, m2 = q[0], q[1]
        M = m1 + m2
        out[0] = (m1 * m2) ** (mp.mpf(3) / 5) / M ** (mp.mpf(1) / 5)
        out[1] = m1 * m2 / M ** 2
    if basis & CHI_SA:
        out[9], out[10] = q[9] + q[10], q[9] - q[10]
    if basis & LAMBDA_TILDE and P >= 13:
        a, b, c, d = _tidal_coeffs(out[1])
        S, D = mp.lu_solve(mp.matrix([[a, b], [c, d]]), mp.matrix([q[11], q[12]]))
        out[11], out[12] = (S + D) / 2, (S - D) / 2
    return out


def jacobian(par, basis, dps: int = 40) -> np.ndarray:
    """J[i][a] = d native_i / d new_a at the event (numerical, dps digits)."""
    P = len(par)
    with mp.workdps(dps):
        q0 = new_parameters(par, basis)
        J = np.zeros((P, P))
        for a in range(P):
            def f(x, a=a):
                q = list(q0)
                q[a] = x
                return native_from_new(q, basis)
            h = mp.mpf(10) ** (-dps // 3) * max(1, abs(q0[a]))
            fp, fm = f(q0[a] + h), f(q0[a] - h)
            fp2, fm2 = f(q0[a] + 2 * h), f(q0[a] - 2 * h)
            for i in range(P):
                J[i, a] = float((8 * (fp[i] - fm[i]) - (fp2[i] - fm2[i])) / (12 * h))
    return J


def fisher_basis(fisher: np.ndarray, par: np.ndarray, basis: int, dps: int = 40) -> np.ndarray:
    """Gamma'[P][P][N] = J^T Gamma J per event; par[P_par][N] native parameters
    (rows beyond P ignored)."""
    P, _, N = fisher.shape
    out = np.zeros_like(fisher)
    for e in range(N):
        J = jacobian(par[:P, e], basis, dps)
        with mp.workdps(dps):
            G = mp.matrix(fisher[:, :, e].tolist())
            Jm = mp.matrix(J.tolist())
            R = Jm.T * G * Jm
            out[:, :, e] = np.array([[float(R[i, j]) for j in range(P)] for i in range(P)])
    return out

"""GPU: the covariance manipulations and the sky area (gwf_covariance,
sec. 4.1-4.2) against the oracle's mpmath epilogue on the same Fisher
matrices.

Tolerances as for the inversion: max(1e-9, 1e3 kappa u) relative for the
condition number, sigma and the normalised covariance, u = 2^-53, kappa the
condition number of the matrix that is inverted.  The sky area takes the
square root of C_tt C_pp - C_tp^2, whose relative error is that of the
entries times (C_tt C_pp + C_tp^2) / det; half of that enters the area.
"""
import math

import numpy as np
import pytest

from paper_2207_06910_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53
# the paper's worked example: spins fixed, a Gaussian prior of variance
# 2 pi^2 on the angles, the 90% region in square degrees; here the tidal
# deformabilities are marginalised over as well
FIXED = [9, 10]
ANGLES = [3, 4, 5, 6, 8]
PRIOR = {i: 1.0 / (2.0 * math.pi ** 2) for i in ANGLES}
MARG = [11, 12]


@pytest.fixture(scope="module")
def lib():
    from paper_2207_06910_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    binding.load()
    return binding


def _gpu(lib, F, theta=None, **kw):
    Ft = torch.as_tensor(np.ascontiguousarray(F), device="cuda")
    th = None if theta is None else torch.as_tensor(np.ascontiguousarray(theta, dtype=np.float64), device="cuda")
    r = lib.covariance(Ft, theta=th, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def _compare(g, ref, sky=True):
    assert np.array_equal(g["status"], ref["status"])
    assert list(g["out"]) == list(ref["out"])
    ok = ref["status"] == 0
    kap = ref["cond"]
    tol = np.maximum(1e-9, 1e3 * kap * U)
    assert np.all(np.abs(g["cond"] / kap - 1) <= tol)
    relsig = np.abs(g["sigma"][:, ok] / ref["sigma_out"][:, ok] - 1).max(axis=0)
    assert np.all(relsig <= tol[ok]), (relsig, tol[ok])
    dc = np.sqrt(np.einsum("iie->ie", ref["cov_out"][:, :, ok]))
    cerr = (np.abs(g["cov"][:, :, ok] - ref["cov_out"][:, :, ok]) / (dc[:, None, :] * dc[None, :, :])).max(axis=(0, 1))
    assert np.all(cerr <= tol[ok])
    assert np.all(g["inv_err"][ok] >= 0) and np.all(np.isnan(g["inv_err"][~ok]))
    if sky:
        C = ref["cov"]
        it, ip = list(ref["keep"]).index(3), list(ref["keep"]).index(4)
        ctt, cpp, ctp = C[it, it], C[ip, ip], C[it, ip]
        amp = (np.abs(ctt * cpp) + ctp ** 2) / (ctt * cpp - ctp ** 2)
        serr = np.abs(g["sky"][ok] / ref["sky"][ok] - 1)
        assert np.all(serr <= tol[ok] * amp[ok]), (serr, tol[ok] * amp[ok])
        assert np.all(np.isnan(g["sky"][~ok]))


def test_epilogue_against_oracle(lib, orc):
    """BNS Fisher matrices of the oracle: spins fixed, priors on the angles,
    tides marginalised, 90% sky area in square degrees and in steradians."""
    wl = synth.bns1e4(n=12).with_npts(2500)
    F = orc.fisher(wl)["fisher"]
    theta = wl.par[3]
    for units in ("SqDeg", "Sterad"):
        g = _gpu(lib, F, theta, fixed=FIXED, prior=PRIOR, marg=MARG, units=units)
        ref = orc.covariance_epilogue(F, fixed=FIXED, prior=PRIOR, marg=MARG, theta=theta, units=units)
        _compare(g, ref)
    # 50% level, nothing fixed, only a prior
    g = _gpu(lib, F, theta, prior={2: 1e-2}, sky_level=50.0)
    ref = orc.covariance_epilogue(F, prior={2: 1e-2}, theta=theta, perc_level=50.0)
    _compare(g, ref)


def test_identity_options_equal_invert(lib, orc):
    """No manipulation: every output bit equals gwf_invert's."""
    wl = synth.bns1e4(n=64).with_npts(800)
    F = torch.as_tensor(orc.fisher(wl)["fisher"], device="cuda")
    a = lib.invert(F)
    b = lib.covariance(F)
    torch.cuda.synchronize()
    for k in ("cov", "sigma", "cond", "inv_err", "logdet", "status"):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.array_equal(x, y, equal_nan=x.dtype.kind == "f"), k


def test_known_inverses(lib):
    """Matrices A with set spectra (kappa <= 1e3 after normalisation): fixing
    S leaves inv(A[~S, ~S]); a prior adds to the diagonal first;
    marginalising keeps the block of that inverse."""
    rng = np.random.default_rng(8)
    P, n = 11, 40
    F = np.zeros((P, P, n))
    for e in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(P, P)))
        A = (Q * np.geomspace(1.0, 1e3, P)) @ Q.T
        A = 0.5 * (A + A.T)
        s = 10 ** rng.uniform(-2, 2, P)
        F[:, :, e] = A * np.outer(s, s)
    fixed, marg, prior = [1, 7], [0, 9], {2: 0.5, 4: 3.0}
    keep = [i for i in range(P) if i not in fixed]
    out = [i for i in keep if i not in marg]
    g = _gpu(lib, F, fixed=fixed, marg=marg, prior=prior)
    assert g["out"] == out
    for e in range(n):
        Fk = F[np.ix_(keep, keep, [e])][:, :, 0].copy()
        for i, v in prior.items():
            Fk[keep.index(i), keep.index(i)] += v
        dk = np.sqrt(np.diag(Fk))                      # normalised: kappa <= 1e3, FP64 inverse to ~1e-13
        C = np.linalg.inv(Fk / np.outer(dk, dk)) / np.outer(dk, dk)
        pos = [keep.index(i) for i in out]
        ref = C[np.ix_(pos, pos)]
        d = np.sqrt(np.diag(ref))
        assert np.max(np.abs(g["cov"][:, :, e] - ref) / np.outer(d, d)) < 1e-11
        np.testing.assert_allclose(g["sigma"][:, e], d, rtol=1e-11)


def test_full_catalogue_sampled_against_oracle(lib, orc):
    """The 10^4-event BNS catalogue's Fisher matrices from the batched plan
    (the benchmark configuration), the paper's example manipulations on all
    of them; sampled events against the oracle's epilogue of the same
    matrices; the sky area is finite and positive wherever the inversion
    succeeded."""
    wl = synth.bns1e4()
    dw = lib.DeviceWorkload(wl)
    plan = lib.Plan(dw, chunk=16384, use_graph=False)
    F = plan.run()["fisher"]
    theta = dw.par[3].contiguous()
    r = lib.covariance(F, theta=theta, fixed=FIXED, prior=PRIOR, marg=MARG)
    torch.cuda.synchronize()
    st = r["status"].cpu().numpy()
    sky = r["sky"].cpu().numpy()
    ok = st == 0
    assert ok.mean() > 0.95
    assert np.all(np.isfinite(sky[ok]) & (sky[ok] > 0))
    idx = np.random.default_rng(5).choice(wl.n, 8, replace=False)
    Fs = F.cpu().numpy()[:, :, idx]
    ref = orc.covariance_epilogue(Fs, fixed=FIXED, prior=PRIOR, marg=MARG, theta=wl.par[3][idx])
    g = {k: (v.cpu().numpy()[..., idx] if hasattr(v, "cpu") else v) for k, v in r.items()}
    _compare(g, ref)
    plan.close()


# ------------------------------------------------------------ SVD inversions and eigen-decomposition
def _spectra(rng, P, n, lam_fn):
    F = np.zeros((P, P, n))
    for e in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(P, P)))
        A = (Q * lam_fn(e)) @ Q.T
        A = 0.5 * (A + A.T)
        s = 10 ** rng.uniform(-2, 2, P)
        F[:, :, e] = A * np.outer(s, s)
    return F


def _cov_close(g, ref, ok, tol):
    dc = np.sqrt(np.abs(np.einsum("iie->ie", ref["cov"][:, :, ok])))
    cerr = (np.abs(g["cov"][:, :, ok] - ref["cov"][:, :, ok]) / (dc[:, None, :] * dc[None, :, :])).max(axis=(0, 1))
    assert np.all(cerr <= tol[ok]), (cerr, tol[ok])


def test_svd_methods_against_oracle(lib, orc):
    """'svd' (plain and truncated) and 'svd_reg' on BNS Fisher matrices
    against the oracle's mpmath SVD inverses of the same matrices, within
    max(1e-9, 1e3 kappa u); 'cho_svd' equals 'cho' where the Cholesky works."""
    wl = synth.bns1e4(n=12).with_npts(2500)
    F = orc.fisher(wl)["fisher"]
    for method, trunc in (("svd", False), ("svd", True), ("svd_reg", False)):
        g = _gpu(lib, F, method=method, truncate=trunc)
        ref = orc.covariance(F, method=method, truncate=trunc)
        assert np.array_equal(g["status"], ref["status"]), method
        ok = ref["status"] == 0
        kap = ref["cond"]
        tol = np.maximum(1e-9, 1e3 * kap * U)
        _cov_close(g, ref, ok, tol)
        assert np.all(g["inv_err"][ok] >= 0)
    a = _gpu(lib, F, method="cho")
    b = _gpu(lib, F, method="cho_svd")
    pd = a["status"] == 0
    for k in ("cov", "sigma", "logdet", "cond", "inv_err"):
        assert np.array_equal(a[k][..., pd], b[k][..., pd]), k


def test_svd_fallback_on_indefinite_matrices(lib, orc):
    """Matrices with negative eigenvalues (positive diagonal): 'cho' flags
    them NOT_PD with NaN outputs; 'cho_svd' inverts them by SVD (status 32,
    the exact inverse within max(1e-9, 1e3 kappa u), ln det NaN); positive
    definite ones in the same launch keep the Cholesky result."""
    rng = np.random.default_rng(31)
    P, n = 9, 24

    def lam(e):
        v = np.geomspace(0.1, 100.0, P)
        if e % 3 == 0:
            v[[0, 3]] *= -1.0
        return v
    F = _spectra(rng, P, n, lam)
    F[np.arange(P), np.arange(P), :] = np.abs(F[np.arange(P), np.arange(P), :]) + 1e-3
    g0 = _gpu(lib, F, method="cho")
    g1 = _gpu(lib, F, method="cho_svd")
    ref = orc.covariance(F, method="cho_svd")
    assert np.array_equal(g1["status"], ref["status"])
    svd = ref["status"] == 32
    assert svd.sum() >= 4 and np.all(g0["status"][svd] == 2) and np.all(np.isnan(g0["sigma"][:, svd]))
    kap = ref["cond"]
    tol = np.maximum(1e-9, 1e3 * kap * U)
    _cov_close(g1, ref, np.ones(n, bool), tol)
    neg = np.einsum("iie->ie", ref["cov"]) < 0
    assert np.array_equal(np.isnan(g1["sigma"]), neg)
    assert np.all(np.isnan(g1["logdet"][svd])) and np.all(np.isfinite(g1["logdet"][~svd]))


def test_logdet_where_the_svd_replaces_a_failed_cholesky(lib):
    """Positive-definite matrices (by their 50-digit eigenvalues) at kappa
    ~1e16-1e19, one eigenvalue near the FP64 rounding level of the others,
    so that the FP64 Cholesky fails on some of them: where 'cho_svd' takes
    the SVD (status 32) and 'svd' likewise falls back from its Cholesky, ln
    det Gamma comes from the singular values and must equal mpmath's ln det.
    The scales s_i (1e3-1e6) make |ln det| about 200-300, so a factor of two
    would miss by that much, while the smallest singular value of a matrix at
    kappa carries a relative error up to ~1e3 kappa u: the tolerance is
    1 + ln(1 + 1e3 kappa u)."""
    mp = pytest.importorskip("mpmath")
    rng = np.random.default_rng(1906)
    P, n = 13, 160
    F = np.zeros((P, P, n))
    for e in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(P, P)))
        lam = np.geomspace(1.0, 0.05, P)
        lam[-1] = 10.0 ** -rng.uniform(16.0, 18.5)
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
        d = np.sqrt(np.diag(A))
        A = A / np.outer(d, d)
        sc = 10 ** rng.uniform(3, 6, P)
        F[:, :, e] = A * np.outer(sc, sc)
    ldr = np.full(n, np.nan)
    kap = np.full(n, np.inf)
    with mp.workdps(50):
        for e in range(n):
            M = mp.matrix(F[:, :, e].tolist())
            dn = [mp.sqrt(M[i, i]) for i in range(P)]
            Mh = mp.matrix(P, P)
            for i in range(P):
                for j in range(P):
                    Mh[i, j] = M[i, j] / (dn[i] * dn[j])
            ev = mp.eigsy(Mh, eigvals_only=True)
            if all(x > 0 for x in ev):
                ldr[e] = float(mp.log(mp.det(M)))
                kap[e] = float(max(ev) / min(ev))
    pd = np.isfinite(ldr)
    assert pd.sum() >= 20
    for method in ("cho_svd", "svd"):
        g = _gpu(lib, F, method=method)
        g0 = _gpu(lib, F, method="cho")
        fell = (g0["status"] == 2) & pd & np.isfinite(g["logdet"])
        assert fell.sum() >= 3, f"{method}: only {fell.sum()} positive-definite matrices took the SVD"
        tol = 1.0 + np.log1p(1e3 * kap[fell] * U)
        err = np.abs(g["logdet"][fell] - ldr[fell])
        assert np.all(err <= tol), (method, err, ldr[fell])
        print(f"{method}: {fell.sum()} positive-definite matrices by SVD, |ln det| "
              f"{np.abs(ldr[fell]).min():.0f}-{np.abs(ldr[fell]).max():.0f}, max error {err.max():.2e}")
        if method == "cho_svd":
            assert np.all(g["status"][fell] == 32)
        # where the FP64 Cholesky worked, both methods keep its ln det
        chol = g0["status"] == 0
        assert np.array_equal(g["logdet"][chol], g0["logdet"][chol])


def test_eigen_decomposition_against_oracle(lib, orc):
    """Eigenvalues (ascending) and eigenvectors of the normalised matrices
    against mpmath's: well-separated spectra, both signs, the sign
    convention of the eigenvectors; with fixed parameters the decomposition
    is of the kept matrix."""
    rng = np.random.default_rng(12)
    P, n = 11, 16
    F = _spectra(rng, P, n, lambda e: np.linspace(1.0, 11.0, P) * (1 if e % 2 else -1) ** (np.arange(P) < 2))
    g = _gpu(lib, F, eigen=True, method="cho_svd")
    val, vec = orc.eigen(F)
    scale = np.abs(val).max(axis=0)
    assert np.max(np.abs(g["eigval"] - val) / scale) < 1e-13
    assert np.max(np.abs(g["eigvec"] - vec)) < 1e-12
    fixed = [2, 7]
    keep = [i for i in range(P) if i not in fixed]
    g = _gpu(lib, F, eigen=True, fixed=fixed)
    val, vec = orc.eigen(np.ascontiguousarray(F[np.ix_(keep, keep)]))
    assert np.max(np.abs(g["eigval"] - val) / np.abs(val).max(axis=0)) < 1e-12
    assert np.max(np.abs(g["eigvec"] - vec)) < 1e-10


# ------------------------------------------------------------ double-double Cholesky
def test_double_double_cholesky_against_oracle(lib, orc):
    """'cho_dd' (the Cholesky inversion in double-double, the counterpart of
    the paper's arbitrary-precision inversion) against the oracle's 50-digit
    inverse of the same FP64 matrices: on BNS Fisher matrices and on
    synthetic spectra up to kappa ~ 1e18, within max(1e-14, 1e3 kappa 2^-104)
    of the normalised covariance, far inside the FP64 Cholesky's
    1e3 kappa 2^-53 (which the worst of these exceed); the epilogue (fixed
    parameters, priors, marginalisation, sky area) on top of it as for
    'cho'."""
    mp = pytest.importorskip("mpmath")
    UD = 2.0 ** -104
    wl = synth.bns1e4(n=12).with_npts(2500)
    F = orc.fisher(wl)["fisher"]
    rng = np.random.default_rng(41)
    P = 13
    S = _spectra(rng, P, 12, lambda e: np.geomspace(1.0, 10.0 ** (6 + e), P))
    for M in (F, S):
        g = _gpu(lib, M, method="cho_dd")
        ref = orc.covariance(M, method="cho")
        assert np.array_equal(g["status"], ref["status"])
        ok = ref["status"] == 0
        assert ok.sum() >= 10
        kap = ref["cond"]
        assert np.all(np.abs(g["cond"][ok] / kap[ok] - 1) <= np.maximum(1e-9, 1e3 * kap[ok] * U))
        tol = np.maximum(1e-14, 1e3 * kap * UD)
        _cov_close(g, ref, ok, tol)
        rels = np.abs(g["sigma"][:, ok] / np.sqrt(np.einsum("iie->ie", ref["cov"][:, :, ok])) - 1)
        assert np.all(rels <= tol[ok])
        with mp.workdps(50):
            ldr = np.array([float(mp.log(mp.det(mp.matrix(M[:, :, e].tolist())))) for e in np.flatnonzero(ok)])
        assert np.all(np.abs(g["logdet"][ok] - ldr) <= 1e-13 * np.maximum(1.0, np.abs(ldr)))
        assert np.all(g["inv_err"][ok] >= 0)
    # the FP64 Cholesky misses the double-double bound on the worst spectra
    g64 = _gpu(lib, S, method="cho")
    ref = orc.covariance(S, method="cho")
    dc = np.sqrt(np.einsum("iie->ie", ref["cov"]))
    e64 = (np.abs(g64["cov"] - ref["cov"]) / (dc[:, None, :] * dc[None, :, :])).max(axis=(0, 1))
    assert e64.max() > 1e-12
    # the epilogue on the double-double inverse
    g = _gpu(lib, F, theta=wl.par[3], fixed=FIXED, prior=PRIOR, marg=MARG, method="cho_dd")
    ref = orc.covariance_epilogue(F, fixed=FIXED, prior=PRIOR, marg=MARG, theta=wl.par[3])
    _compare(g, ref)

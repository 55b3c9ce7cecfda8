"""GPU parity: libgwf (through its C ABI) against the CPU oracle.

Tolerances (plain FP64 form): SNR relative error <= 1e-12; Fisher elements
|dGamma_ij| / sqrt(Gamma_ii Gamma_jj) <= 1e-9 (the paper's own normalisation,
sec. 4.1); covariance and sigma against mpmath on the SAME Fisher matrix
within max(1e-9, 1e3 kappa u) relative, u = 2^-53, the backward-stability
bound of a Cholesky inversion at condition number kappa.
"""
import numpy as np
import pytest

from paper_2207_06910_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def lib():
    from paper_2207_06910_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    binding.load()
    return binding


def _run(lib, wl, **kw):
    dw = lib.DeviceWorkload(wl)
    r = lib.fisher(dw, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def _fisher_err(F, Fref):
    d = np.sqrt(np.abs(np.einsum("iie->ie", Fref)))
    return np.abs(F - Fref) / (d[:, None, :] * d[None, :, :])


def _assert_parity(g, ref, snr_tol=1e-12, f_tol=1e-9):
    np.testing.assert_array_equal(g["status"], 0)
    rel = np.abs(g["snr"] / ref["snr"] - 1)
    assert rel.max() <= snr_tol, f"SNR rel err {rel.max():.3e}"
    err = _fisher_err(g["fisher"], ref["fisher"])
    assert err.max() <= f_tol, f"Fisher err {err.max():.3e} at {np.unravel_index(err.argmax(), err.shape)}"
    assert np.array_equal(g["fisher"], g["fisher"].transpose(1, 0, 2))
    return rel.max(), err.max()


def test_bbh100_single_detector(lib, orc):
    """100 BBH events, one L detector at the H1 site, no Earth rotation,
    1000-point grids from 10 Hz to the cut frequency, 11 parameters."""
    wl = synth.bbh100()
    g = _run(lib, wl, per_ifo_snr=True)
    ref = orc.fisher(wl)
    s, f = _assert_parity(g, ref)
    print(f"bbh100: SNR {s:.2e}, Fisher {f:.2e}")
    np.testing.assert_allclose(g["snr_ifo"][0], g["snr"], rtol=1e-13)


def test_bns_network_full_grids(lib, orc):
    """BNS events of the 10^4 catalogue with their full 2000-20000-point grids
    from 2 Hz, triangle + two L sites, Earth rotation, tides (13 parameters);
    the shortest and the longest grids of the catalogue are included."""
    full = synth.bns1e4()
    idx = np.unique(np.r_[np.argmin(full.npts), np.argmax(full.npts),
                          np.random.default_rng(5).choice(full.n, 10, replace=False)])
    wl = full.subset(idx)
    g = _run(lib, wl, per_ifo_snr=True)
    ref = orc.fisher(wl)
    s, f = _assert_parity(g, ref)
    print(f"bns full grids {wl.npts.min()}-{wl.npts.max()}: SNR {s:.2e}, Fisher {f:.2e}")
    np.testing.assert_allclose(g["snr_ifo"], ref["snr_ifo"], rtol=1e-12)


@pytest.mark.parametrize("flags", [0, synth.FLAG_EARTH_ROT, synth.FLAG_TIDAL,
                                   synth.FLAG_TIDAL | synth.FLAG_EARTH_ROT])
def test_ragged_grids_and_flag_combinations(lib, orc, flags):
    """Grid lengths around the 256-lane stride (2, 3, 255, 256, 257, 511,
    513, 1000) in one launch, every combination of rotation and tides."""
    wl = synth.bns1e4(n=8)
    wl.npts = np.array([2, 3, 255, 256, 257, 511, 513, 1000], dtype=np.int32)
    wl.flags = flags
    g = _run(lib, wl)
    ref = orc.fisher(wl)
    _assert_parity(g, ref)


def test_single_event_explicit_fmax_and_tc(lib, orc):
    wl = synth.bns1e4(n=1).with_npts(700)
    wl.fmin = np.array([5.0])
    wl.fmax = np.array([640.0])
    wl.tc_s = np.array([1.2e9])             # enters only the waveform phase
    g = _run(lib, wl)
    ref = orc.fisher(wl)
    _assert_parity(g, ref)


def test_invalid_events_flagged_and_isolated(lib, orc):
    wl = synth.bns1e4(n=6).with_npts(600)
    wl.par[1, 0] = 0.26                     # eta > 1/4
    wl.par[2, 1] = 0.0                      # dL = 0
    wl.par[4, 2] = np.inf                   # phi
    wl.npts[3] = 1                          # too short a grid
    g = _run(lib, wl)
    np.testing.assert_array_equal(g["status"][:4], [1, 1, 8, 1])
    assert np.all(g["fisher"][:, :, :4] == 0) and np.all(g["snr"][:4] == 0)
    ref = orc.fisher(wl.subset([4, 5]))
    sub = {k: v[..., 4:] for k, v in g.items()}
    _assert_parity(sub, ref)


def test_snr_threshold_skips_fisher(lib, orc):
    wl = synth.bns1e4(n=10).with_npts(800)
    ref = orc.fisher(wl)
    th = float(np.median(ref["snr"]))
    g = _run(lib, wl, snr_th=th)
    below = ref["snr"] <= th
    assert np.all(g["status"][below] == 16) and np.all(g["status"][~below] == 0)
    assert np.all(g["fisher"][:, :, below] == 0)
    np.testing.assert_allclose(g["snr"], ref["snr"], rtol=1e-12)
    err = _fisher_err(g["fisher"][:, :, ~below], ref["fisher"][:, :, ~below])
    assert err.max() <= 1e-9


def test_snr_entry_point(lib, orc):
    wl = synth.bns1e4(n=7).with_npts(3000)
    dw = lib.DeviceWorkload(wl)
    r = lib.snr(dw, per_ifo=True)
    torch.cuda.synchronize()
    ref = orc.fisher(wl, want_fisher=False)
    np.testing.assert_allclose(r["snr"].cpu().numpy(), ref["snr"], rtol=1e-12)
    np.testing.assert_allclose(r["snr_ifo"].cpu().numpy(), ref["snr_ifo"], rtol=1e-12)


def test_bitwise_reproducible(lib):
    wl = synth.bns1e4(n=16).with_npts(4000)
    a = _run(lib, wl)
    b = _run(lib, wl)
    assert np.array_equal(a["fisher"], b["fisher"]) and np.array_equal(a["snr"], b["snr"])


def test_full_catalogue_sampled_and_invariants(lib, orc):
    """The whole 10^4-event BNS catalogue in the benchmark's launch; sampled
    events against the oracle, and for every event the exact identities
    Gamma_dLdL dL^2 = SNR^2, symmetry and a positive diagonal."""
    full = synth.bns1e4()
    g = _run(lib, full)
    assert np.all(g["status"] == 0)
    idx = np.random.default_rng(11).choice(full.n, 6, replace=False)
    ref = orc.fisher(full.subset(idx))
    sub = {k: v[..., idx] for k, v in g.items()}
    _assert_parity(sub, ref)
    F = g["fisher"]
    np.testing.assert_allclose(F[2, 2] * full.par[2] ** 2, g["snr"] ** 2, rtol=1e-12)
    assert np.all(np.einsum("iie->ie", F) > 0)


# ----------------------------------------------------------------- inversion
def _invert_gpu(lib, F, status=None, cond_max=1e50):
    Ft = torch.as_tensor(np.ascontiguousarray(F), device="cuda")
    st = None if status is None else torch.as_tensor(status, device="cuda")
    r = lib.invert(Ft, st, cond_max=cond_max)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def test_inversion_against_mpmath_same_fisher(lib, orc):
    """GPU inversion of the oracle's Fisher matrices against a 50-digit
    mpmath inversion of the same matrices."""
    wl = synth.bns1e4(n=12).with_npts(2500)
    F = orc.fisher(wl)["fisher"]
    for P in (13, 9):                       # also a sub-block (fixed parameters)
        Fp = np.ascontiguousarray(F[:P, :P])
        g = _invert_gpu(lib, Fp)
        ref = orc.covariance(Fp)
        ok = ref["status"] == 0
        assert np.array_equal(g["status"], ref["status"])
        kap = ref["cond"]
        tol = np.maximum(1e-9, 1e3 * kap * U)
        assert np.all(np.abs(g["cond"] / kap - 1) <= tol)
        relsig = np.abs(g["sigma"][:, ok] / ref["sigma"][:, ok] - 1).max(axis=0)
        assert np.all(relsig <= tol[ok]), (relsig, tol[ok])
        dc = np.sqrt(np.einsum("iie->ie", ref["cov"][:, :, ok]))
        cerr = (np.abs(g["cov"][:, :, ok] - ref["cov"][:, :, ok]) /
                (dc[:, None, :] * dc[None, :, :])).max(axis=(0, 1))
        assert np.all(cerr <= tol[ok])
        assert np.all(g["inv_err"][ok] >= 0)


def test_inversion_well_conditioned_exact(lib):
    """Matrices with known inverses and modest condition numbers: sigma to
    1e-12, condition number to 1e-10, inversion error at rounding level."""
    rng = np.random.default_rng(3)
    P, n = 13, 200
    F = np.zeros((P, P, n))
    Cinv = np.zeros((P, P, n))
    kap = np.zeros(n)
    for e in range(n):
        Q, _ = np.linalg.qr(rng.normal(size=(P, P)))
        lam = np.geomspace(1.0, 10 ** rng.uniform(0, 4), P)
        A = (Q * lam) @ Q.T
        d = np.sqrt(np.diag(A))
        A = A / np.outer(d, d)
        s = 10 ** rng.uniform(-3, 3, P)
        F[:, :, e] = A * np.outer(s, s)
        Cinv[:, :, e] = np.linalg.inv(A) / np.outer(s, s)
        ev = np.linalg.eigvalsh(A)
        kap[e] = ev.max() / ev.min()
    g = _invert_gpu(lib, F)
    assert np.all(g["status"] == 0)
    sig = np.sqrt(np.einsum("iie->ie", Cinv))
    np.testing.assert_allclose(g["sigma"], sig, rtol=1e-11)
    np.testing.assert_allclose(g["cond"], kap, rtol=1e-9)
    # inversion error: the GPU's max|Gamma Cov - 1| against the same quantity
    # in extended precision, within the rounding of an FP64 evaluation
    C = g["cov"].astype(np.longdouble)
    Fl = F.astype(np.longdouble)
    for e in range(n):
        R = Fl[:, :, e] @ C[:, :, e] - np.eye(P, dtype=np.longdouble)
        ref = float(np.abs(R).max())
        scale = float((np.abs(Fl[:, :, e]) @ np.abs(C[:, :, e])).max())
        assert abs(g["inv_err"][e] - ref) <= 4 * P * U * scale


def test_inversion_flags(lib):
    """cond > cond_max -> ILL_COND; not positive definite -> NOT_PD; NaN ->
    NONFINITE; events already flagged INVALID/SKIPPED are left alone."""
    P, n = 5, 5
    F = np.zeros((P, P, n))
    for e in range(n):
        F[:, :, e] = np.eye(P) + 0.1 * np.ones((P, P))
    F[:, :, 1] = np.eye(P)
    F[0, 1, 1] = F[1, 0, 1] = 1.0 - 1e-13    # two nearly parallel rows: kappa ~ 2e13
    F[0, 1, 2] = F[1, 0, 2] = 2.0            # indefinite
    F[3, 3, 3] = np.nan
    status = np.array([0, 0, 0, 0, 16], dtype=np.int32)
    g = _invert_gpu(lib, F, status, cond_max=1e12)
    np.testing.assert_array_equal(g["status"], [0, 4, 2, 8, 16])
    assert np.all(np.isfinite(g["sigma"][:, 0])) and np.all(np.isnan(g["sigma"][:, 1:]))


def test_degenerate_inclinations(lib, orc):
    """Face-on, edge-on and face-away binaries (iota = 0, pi/2, pi, and 1e-6
    off each).  The kernels form the Fisher rows of dL, iota and psi from
    pattern moments whose coefficients (sin iota, cos iota and their
    products) vanish or nearly cancel there.  Both forms match the oracle
    element by element (normalised by sqrt(G_ii G_jj)); where the oracle's
    diagonal entry is exactly zero (the iota row at iota = 0) the GPU's row
    is exactly zero too."""
    wl = synth.bns1e4(n=9).with_npts(900)
    wl.par[5] = np.array([0.0, np.pi / 2, np.pi, 1e-6, np.pi / 2 - 1e-6, np.pi - 1e-6,
                          0.3, 1.3, 2.9])
    ref = orc.fisher(wl)
    dg = np.einsum("iie->ie", ref["fisher"])
    zero = dg == 0.0
    assert zero[5, 0] and zero.sum() == 1          # only the iota row at iota = 0
    d = np.sqrt(np.where(zero, 1.0, np.abs(dg)))
    dw = lib.DeviceWorkload(wl)
    plain = _run(lib, wl)
    plan = lib.Plan(dw, chunk=512)
    batched = {k: v.cpu().numpy() for k, v in plan.run().items()}
    torch.cuda.synchronize()
    plan.close()
    for name, g in (("plain", plain), ("batched", batched)):
        np.testing.assert_array_equal(g["status"], 0)
        rel = np.abs(g["snr"] / ref["snr"] - 1).max()
        assert rel <= 1e-12, f"{name}: SNR rel err {rel:.3e}"
        err = np.abs(g["fisher"] - ref["fisher"]) / (d[:, None, :] * d[None, :, :])
        assert err.max() <= 1e-9, f"{name}: Fisher err {err.max():.3e} at {np.unravel_index(err.argmax(), err.shape)}"
        assert np.all(g["fisher"][5, :, 0] == 0.0) and np.all(g["fisher"][:, 5, 0] == 0.0), name
        print(f"degenerate inclinations, {name}: SNR {rel:.2e}, Fisher {err.max():.2e}")

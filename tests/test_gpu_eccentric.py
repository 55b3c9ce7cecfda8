"""GPU: moderate eccentricity (sec. 2.2 is_eccentric; e0 at a reference
frequency, sec. 2.1; e0 the Fisher matrix's last row, sec. 3.2) in the
Fisher (plain, batched FP64 and mixed, static workspace), strain, strain
derivative, adjoint and inversion kernels, against the oracle.

Inputs: BNS events of the benchmark catalogue and BBH events of the small
configuration, with seeded e0 ~ U(0.01, 0.1) given at the grid's first
frequency or at 10 Hz.  Bars as for the circular forms: SNR 1e-12, Fisher
1e-9 of sqrt(G_ii G_jj), strain and derivatives within their phase-error
bounds (test_gpu_waveform, test_gpu_waveform_deriv), the adjoint 1e-10 of
its size; with e0 = 0 the eccentric Fisher matrix equals the circular one
bit for bit with a zero e0 row."""
import numpy as np
import pytest

from paper_2207_06910_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53
ECC = synth.FLAG_ECCENTRIC


@pytest.fixture(scope="module")
def lib():
    from paper_2207_06910_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    binding.load()
    return binding


def _bns(n, seed=23, npts=None, f_ref=None):
    full = synth.bns1e4()
    rng = np.random.default_rng(seed)
    wl = full.subset(np.sort(rng.choice(full.n, n, replace=False)))
    if npts is not None:
        wl = wl.with_npts(npts)
    return wl.with_eccentricity(rng.uniform(0.01, 0.1, n), f_ref)


def _np(r):
    return {k: v.cpu().numpy() for k, v in r.items() if hasattr(v, "cpu")}


def _check(g, ref, snr_tol=1e-12, f_tol=1e-9):
    assert np.all(g["status"] == 0), g["status"]
    rel = np.abs(g["snr"] / ref["snr"] - 1).max()
    assert rel <= snr_tol, rel
    d = np.sqrt(np.abs(np.einsum("iie->ie", ref["fisher"])))
    err = (np.abs(g["fisher"] - ref["fisher"]) / (d[:, None, :] * d[None, :, :])).max()
    assert err <= f_tol, err
    return rel, err


@pytest.mark.parametrize("f_ref", [None, 10.0])
def test_eccentric_fisher_bns_full_grids(lib, orc, f_ref):
    """14 parameters (tides, rotation, e0 last) on full 2000-20000-point
    grids; e0 given at the grid start (2 Hz) or at 10 Hz."""
    wl = _bns(6, f_ref=f_ref)
    g = _np(lib.fisher(lib.DeviceWorkload(wl)))
    assert g["fisher"].shape[0] == 14
    rel, err = _check(g, orc.fisher(wl))
    assert np.all(g["fisher"][13, 13] > 0)
    print(f"eccentric BNS (f_ref {f_ref}): SNR {rel:.2e}, Fisher {err:.2e}")


def test_eccentric_fisher_bbh_no_rotation(lib, orc):
    """12 parameters (no tides, e0 last) on one L site without rotation."""
    wl = synth.bbh100(n=10)
    wl = wl.with_eccentricity(np.random.default_rng(4).uniform(0.02, 0.1, wl.n))
    g = _np(lib.fisher(lib.DeviceWorkload(wl)))
    assert g["fisher"].shape[0] == 12
    _check(g, orc.fisher(wl))


def test_eccentric_zero_is_circular_bit_for_bit(lib):
    """With e0 = 0 the eccentric kernels add exact zeros: the 13 x 13 block
    equals the circular kernels' matrix bit for bit and the e0 row is 0."""
    full = synth.bns1e4(n=5).with_npts(1500)
    circ = _np(lib.fisher(lib.DeviceWorkload(full)))
    ecc = _np(lib.fisher(lib.DeviceWorkload(full.with_eccentricity(0.0))))
    assert np.array_equal(ecc["fisher"][:13, :13], circ["fisher"])
    assert np.all(ecc["fisher"][13] == 0) and np.all(ecc["fisher"][:, 13] == 0)
    assert np.array_equal(ecc["snr"], circ["snr"])


@pytest.mark.parametrize("mixed", [False, True])
def test_eccentric_plan_and_static(lib, orc, mixed):
    wl = _bns(8, seed=5)
    dw = lib.DeviceWorkload(wl)
    plan = lib.Plan(dw, chunk=4096, mixed=mixed)
    r = _np(plan.run())
    plan.close()
    _check(r, orc.fisher(wl), 5e-7 if mixed else 1e-12, 1e-6 if mixed else 1e-9)
    st = _np(lib.fisher_static(dw, chunk=4096, mixed=mixed))
    for k in ("fisher", "snr", "status"):
        assert np.array_equal(st[k], r[k]), k


def test_eccentric_invalid_values_flagged(lib):
    wl = _bns(4, npts=600)
    wl.ecc[:] = [-0.1, 1.0, np.nan, 0.05]
    g = _np(lib.fisher(lib.DeviceWorkload(wl)))
    np.testing.assert_array_equal(g["status"], [1, 1, 8, 0])
    assert np.all(g["fisher"][:, :, :3] == 0)


def _eps_strain(orc, wl, offsets, total):
    eps = np.full(total, np.nan)
    for e in range(wl.n):
        p = np.concatenate([wl.par[:, e], [wl.ecc[e], 0.0 if wl.f_ref_ecc is None else wl.f_ref_ecc[e]]])
        f, _ = orc.grid(wl.fmin[e], orc.cut_frequency(p[0], p[1]), int(wl.npts[e]))
        psi, tau = orc.phase_tau(p, f, wl.flags)
        eps[offsets[e]:offsets[e] + wl.npts[e]] = 1e-13 + 64 * U * (np.abs(psi) + 2 * np.pi * f * (np.abs(tau) + 0.03))
    return eps


def test_eccentric_strain_and_derivatives(lib, orc):
    """The strain with the eccentric phase, and its 14 derivatives, against
    the oracle within the phase-error bounds of the circular tests."""
    wl = _bns(3, npts=800, f_ref=12.0)
    npts = wl.npts.astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(npts)[:-1]])
    total = int(npts.sum())
    dw = lib.DeviceWorkload(wl)
    off = torch.as_tensor(offsets, device="cuda")
    h = lib.waveform(dw, offsets=off, total=total)["h"].cpu().numpy()
    dh = lib.waveform_deriv(dw, offsets=off, total=total)["dh"].cpu().numpy()
    href = orc.waveform(wl, offsets, total)
    dref = orc.waveform_derivs(wl, offsets, total)
    eps = _eps_strain(orc, wl, offsets, total)
    tol = np.abs(href) * eps[None, :] + 1e-13 * np.abs(href).max(axis=0)[None, :]
    assert np.all(np.abs(h - href) <= tol), (np.abs(h - href) / tol).max()
    assert dh.shape[0] == 14
    tol = np.abs(dref) * eps[None, None, :] + 1e-11 * np.abs(dref).max(axis=1, keepdims=True)
    worst = (np.abs(dh - dref) / tol).max()
    assert worst <= 1.0, worst
    # the e0 row is nonzero where e0 is
    assert np.abs(dh[13]).max() > 0


def test_eccentric_inversion_same_fisher(lib, orc):
    """14 x 14 inversions of the oracle's eccentric Fisher matrices against
    mpmath on the same matrices, within max(1e-9, 1e3 kappa u)."""
    wl = _bns(6, seed=9, npts=2500)
    F = orc.fisher(wl)["fisher"]
    g = lib.covariance(torch.as_tensor(F, device="cuda"), method="cho_svd")
    g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in g.items()}
    ref = orc.covariance(F, dps=50, method="cho_svd")
    assert np.array_equal(g["status"], ref["status"])
    ok = ref["status"] == 0
    tol = np.maximum(1e-9, 1e3 * ref["cond"] * U)
    rel = np.abs(g["sigma"][:, ok] / ref["sigma"][:, ok] - 1).max(axis=0)
    assert np.all(rel <= tol[ok]), (rel, tol[ok])


def test_eccentric_adjoint(lib, orc):
    """Detector gradients with e0 in the Fisher matrix (Gbar 14 x 14 scaled
    like an inverse Fisher matrix) against the oracle's nested duals."""
    wl = _bns(3, seed=2, npts=600)
    F = orc.fisher(wl)["fisher"]
    d = np.sqrt(np.einsum("iie->ie", F))
    P = F.shape[0]
    gbar = np.random.default_rng(8).normal(size=(P, P, wl.n)) / (d[:, None, :] * d[None, :, :])
    r = lib.fisher_adjoint(lib.DeviceWorkload(wl), torch.as_tensor(gbar, device="cuda"), w_snr=0.3,
                           w_fisher=1.1)
    ge = r["grad_event"].cpu().numpy()
    ns = len(wl.sites)
    tang = [[orc.fisher_tangent(wl, s, m) for m in range(4)] for s in range(ns)]
    dF = np.array([[t["fisher"][1] for t in row] for row in tang])
    dS = np.array([[t["snr2"][1] for t in row] for row in tang])
    S2 = tang[0][0]["snr2"][0]
    Gs = 0.5 * (gbar + gbar.transpose(1, 0, 2))
    ref = 1.1 * np.einsum("ije,smije->esm", Gs, dF) + 0.3 * np.transpose(dS, (2, 0, 1)) / (2 * S2[:, None, None])
    err = np.abs(ge - ref) / np.abs(ref).max(axis=(1, 2), keepdims=True)
    assert err.max() < 1e-10, err.max()

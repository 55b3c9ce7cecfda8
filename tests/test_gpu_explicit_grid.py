"""GPU: explicit frequency grids (GWF_GRID_EXPLICIT) in gwf_snr, gwf_fisher,
gwf_fisher_ifo, gwf_waveform and gwf_waveform_deriv, against the oracle's
explicit-grid sums on the same frequencies.

Tolerances as for the log grids: SNR 1e-12 relative, Fisher 1e-9 of
sqrt(G_aa G_bb); the strain and its derivatives within |ref| eps_k plus a
floor of 1e-13 (strain) or 1e-11 (derivatives) of the point's largest value,
eps_k = 1e-13 + 64 u (|Psi_PN(f_k)| + 2 pi f_k (tau*(f_k) + 0.03 s)).  On the
log grid's own frequencies the explicit path must reproduce the descriptor
path to rounding (the frequencies agree to an ulp or so).
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


def _np(r):
    return {k: v.cpu().numpy() for k, v in r.items()}


def _ferr(F, R):
    d = np.sqrt(np.abs(np.einsum("...iie->...ie", R)))
    return (np.abs(F - R) / (d[..., :, None, :] * d[..., None, :, :])).max()


def _workloads(orc):
    wl = synth.bns1e4().subset(np.arange(3)).with_npts(600)
    fc = [orc.cut_frequency(wl.par[0, e], wl.par[1, e]) for e in range(wl.n)]
    logf = [orc.grid(wl.fmin[e], fc[e], int(wl.npts[e]))[0] for e in range(wl.n)]
    lin = [np.linspace(wl.fmin[e], fc[e], n) for e, n in zip(range(wl.n), (700, 455, 1001))]
    return wl, wl.with_grid_f(logf), wl.with_grid_f(lin)


def _eps(orc, wl, total):
    eps = np.full(total, np.nan)
    off = wl.grid_offsets()
    for e in range(wl.n):
        f = wl.event_grid(e)
        psi, tau = orc.phase_tau(wl.par[:, e], f, wl.flags)
        eps[off[e]:off[e] + wl.npts[e]] = 1e-13 + 64 * U * (np.abs(psi) + 2 * np.pi * f * (np.abs(tau) + 0.03))
    return eps


def test_explicit_log_frequencies_reproduce_descriptors(lib, orc):
    """The log grid's frequencies given explicitly: SNR, Fisher and the
    per-interferometer matrices as on the descriptor grid."""
    wl, wlog, _ = _workloads(orc)
    a = _np(lib.fisher(lib.DeviceWorkload(wl)))
    b = _np(lib.fisher(lib.DeviceWorkload(wlog)))
    np.testing.assert_array_equal(b["status"], 0)
    np.testing.assert_allclose(b["snr"], a["snr"], rtol=1e-13)
    assert _ferr(b["fisher"], a["fisher"]) <= 1e-12
    fi = lib.fisher_ifo(lib.DeviceWorkload(wlog))["fisher_ifo"].cpu().numpy()
    assert _ferr(fi.sum(axis=0), a["fisher"]) <= 1e-12


def test_linear_grids_against_oracle(lib, orc):
    """Linear grids of different lengths: SNR (both entry points), Fisher,
    per-interferometer Fisher, strain and strain derivatives against the
    oracle on the same frequencies."""
    _, _, wl = _workloads(orc)
    dw = lib.DeviceWorkload(wl)
    ref = orc.fisher(wl, per_ifo=True)
    g = _np(lib.fisher(dw))
    np.testing.assert_array_equal(g["status"], 0)
    np.testing.assert_allclose(g["snr"], ref["snr"], rtol=1e-12)
    assert _ferr(g["fisher"], ref["fisher"]) <= 1e-9
    s = lib.snr(dw, per_ifo=True)
    np.testing.assert_allclose(s["snr"].cpu().numpy(), ref["snr"], rtol=1e-12)
    fi = lib.fisher_ifo(dw)["fisher_ifo"].cpu().numpy()
    assert _ferr(fi, ref["fisher_ifo"]) <= 1e-9
    total = int(wl.npts.sum())
    eps = _eps(orc, wl, total)
    h = lib.waveform(dw)["h"].cpu().numpy()
    href = orc.waveform(wl)
    tol = np.abs(href) * eps[None, :] + 1e-13 * np.abs(href).max(axis=0)[None, :]
    assert (np.abs(h - href) / tol).max() <= 1.0
    dh = lib.waveform_deriv(dw)["dh"].cpu().numpy()
    dref = orc.waveform_derivs(wl)
    tol = np.abs(dref) * eps[None, None, :] + 1e-11 * np.abs(dref).max(axis=1, keepdims=True)
    assert (np.abs(dh - dref)[tol > 0] / tol[tol > 0]).max() <= 1.0


def test_invalid_explicit_grids_flagged(lib, orc):
    """A grid whose first frequency is not positive, or whose last is not
    above the first, flags its event invalid (zero outputs) and leaves the
    others as they are; plans refuse explicit grids."""
    _, _, wl = _workloads(orc)
    freqs = [wl.event_grid(e).copy() for e in range(wl.n)]
    freqs[0][0] = 0.0
    freqs[2] = freqs[2][::-1].copy()
    bad = wl.with_grid_f(freqs)
    g = _np(lib.fisher(lib.DeviceWorkload(bad)))
    assert g["status"][0] & 1 and g["status"][2] & 1 and g["status"][1] == 0
    assert np.all(g["fisher"][:, :, [0, 2]] == 0) and np.all(g["snr"][[0, 2]] == 0)
    good = _np(lib.fisher(lib.DeviceWorkload(wl)))
    np.testing.assert_array_equal(g["fisher"][:, :, 1], good["fisher"][:, :, 1])
    with pytest.raises(lib.GwfError):
        lib.Plan(lib.DeviceWorkload(wl))

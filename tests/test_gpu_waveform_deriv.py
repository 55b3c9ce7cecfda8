"""GPU parity of gwf_waveform_deriv (the strain's derivatives with respect
to the Fisher matrix's parameters) against the oracle's dual-number
derivatives of the same strain, and its consistency with gwf_fisher.

Tolerance.  Each derivative is the strain's phase factor times a phase-free
vector D_a; the phase carries the strain's error eps_k (see
test_gpu_waveform), and D_a, a sum of a few terms (the amplitude, pattern
and phase derivatives), carries a few ulp of its largest term.  Per point k,
parameter a and interferometer i the test allows
    |dh_gpu - dh_orc| <= |dh_orc| eps_k + 1e-11 max_i |dh_orc_a,i,k|,
the floor covering those terms' rounding relative to the largest
interferometer's value (a pattern that nearly vanishes at one of them).
The Fisher matrix summed on the host from the GPU's derivatives
(4 Re sum w dh dh^* / S_n) must equal gwf_fisher's to 1e-11 of
sqrt(G_aa G_bb): the same analytic vectors, summed in another order.
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


def _offsets(npts, gap):
    """First column of each event, `gap` unused columns before each event
    and after the last, and the row length."""
    n = np.asarray(npts, dtype=np.int64)
    ends = np.cumsum(n + gap)
    return ends - n, int(ends[-1] + gap)


def _eps(orc, wl, offsets, total):
    eps = np.full(total, np.nan)
    for e in range(wl.n):
        p = wl.par[:, e]
        fmax = orc.cut_frequency(p[0], p[1])
        f, _ = orc.grid(wl.fmin[e], fmax, int(wl.npts[e]))
        psi, tau = orc.phase_tau(p, f, wl.flags)
        tc = 0.0 if wl.tc_s is None else abs(wl.tc_s[e])
        eps[offsets[e]:offsets[e] + wl.npts[e]] = 1e-13 + 64 * U * (np.abs(psi) + 2 * np.pi * f * (tc + np.abs(tau) + 0.03))
    return eps


def _gpu(lib, wl, offsets, total, fill=None):
    dw = lib.DeviceWorkload(wl)
    P = 13 if wl.flags & synth.FLAG_TIDAL else 11
    out = {}
    if fill is not None:
        out["dh"] = torch.full((P, dw.n_ifo, total), fill, dtype=torch.complex128, device="cuda")
    r = lib.waveform_deriv(dw, offsets=torch.as_tensor(offsets, device="cuda"), total=total, out=out)
    torch.cuda.synchronize()
    return r["dh"].cpu().numpy(), r["status"].cpu().numpy()


def _check_against_oracle(orc, wl, dh, offsets, total):
    ref = orc.waveform_derivs(wl, offsets=offsets, total=total)
    eps = _eps(orc, wl, offsets, total)
    used = np.isfinite(eps)
    floor = 1e-11 * np.abs(ref).max(axis=1, keepdims=True)
    err = np.abs(dh - ref)[:, :, used]
    tol = (np.abs(ref) * eps[None, None, :] + floor)[:, :, used]
    assert np.all(err[tol == 0] == 0)          # rows outside a parameter set: exactly zero
    worst = (err[tol > 0] / tol[tol > 0]).max()
    assert worst <= 1.0, f"derivative error {worst:.3f} x tolerance"
    return worst, ref


def _fisher_from(orc, wl, dh, offsets):
    sa = wl.site_array()
    psd = []
    for row in sa:
        psd += [(row[5], row[6])] * (3 if int(row[4]) == synth.SHAPE_T else 1)
    P = dh.shape[0]
    F = np.zeros((P, P, wl.n))
    for e in range(wl.n):
        f, w = orc.grid(wl.fmin[e], orc.cut_frequency(wl.par[0, e], wl.par[1, e]), int(wl.npts[e]))
        for i, (S0, f0) in enumerate(psd):
            S = np.array([orc.psd(S0, f0, x) for x in f])
            d = dh[:, i, offsets[e]:offsets[e] + wl.npts[e]]
            F[:, :, e] += 4.0 * np.real((d * (w / S)) @ d.conj().T)
    return F


def _fisher_close(F, G):
    d = np.sqrt(np.where(np.einsum("iie->ie", G) > 0, np.einsum("iie->ie", G), 1.0))
    return (np.abs(F - G) / (d[:, None, :] * d[None, :, :])).max()


@pytest.mark.parametrize("name", ["bbh100", "bns1e4"])
def test_derivatives_against_oracle_and_fisher(lib, orc, name):
    """One L detector without rotation (11 parameters) and the triangle + two
    L network with rotation and tides (13), ragged grids with gaps between
    events: every derivative against the oracle, the columns between events
    untouched, and the Fisher matrix rebuilt from the derivatives equal to
    gwf_fisher's."""
    if name == "bbh100":
        wl = synth.bbh100().subset(np.arange(5))
    else:
        full = synth.bns1e4()
        wl = full.subset(np.r_[np.argmin(full.npts), 0, 1]).with_npts(600)
        wl.npts = np.array([600, 333, 451], dtype=np.int32)
    offsets, total = _offsets(wl.npts, 7)
    dh, st = _gpu(lib, wl, offsets, total, fill=complex(3.0, -5.0))
    np.testing.assert_array_equal(st, 0)
    worst, ref = _check_against_oracle(orc, wl, dh, offsets, total)
    gap = np.ones(total, bool)
    for e in range(wl.n):
        gap[offsets[e]:offsets[e] + wl.npts[e]] = False
    assert np.all(dh[:, :, gap] == complex(3.0, -5.0))
    dw = lib.DeviceWorkload(wl)
    G = lib.fisher(dw)["fisher"].cpu().numpy()
    F = _fisher_from(orc, wl, dh, offsets)
    err = _fisher_close(F, G)
    assert err <= 1e-11, err
    print(f"{name}: worst derivative error {worst:.3f} x tolerance, Fisher from dh {err:.2e}")


def test_parameter_sets_invalid_events_and_mixed(lib, orc):
    """Rows outside an event's parameter set are zero (the kept rows as
    without a set); an event with invalid parameters is flagged and writes
    nothing; the mixed form is refused."""
    full = synth.mixed1e4(n=200)
    kind = full.meta["kind"]
    idx = np.r_[np.flatnonzero(kind == 0)[:2], np.flatnonzero(kind == 1)[:2]]
    wl = full.subset(idx).with_npts(300)
    offsets, total = _offsets(wl.npts, 0)
    dh, st = _gpu(lib, wl, offsets, total)
    np.testing.assert_array_equal(st, 0)
    _check_against_oracle(orc, wl, dh, offsets, total)
    w0 = wl.subset(np.arange(wl.n))
    w0.par_mask = None
    dh0, _ = _gpu(lib, w0, offsets, total)
    for e in range(wl.n):
        cols = slice(offsets[e], offsets[e] + wl.npts[e])
        for r in range(13):
            if (int(wl.par_mask[e]) >> r) & 1:
                assert np.array_equal(dh[r, :, cols], dh0[r, :, cols])
            else:
                assert np.all(dh[r, :, cols] == 0)
    bad = wl.subset(np.arange(wl.n))
    bad.par[1, 2] = 0.3
    dhb, stb = _gpu(lib, bad, offsets, total, fill=complex(1.0, 1.0))
    assert stb[2] & 1 and np.all(stb[[0, 1, 3]] == 0)
    cols = slice(offsets[2], offsets[2] + wl.npts[2])
    assert np.all(dhb[:, :, cols] == complex(1.0, 1.0))
    dw = lib.DeviceWorkload(wl)
    ev, net, grid, _ = dw.descriptors()
    import ctypes
    off = torch.as_tensor(offsets, device="cuda")
    out = torch.empty((13, dw.n_ifo, total), dtype=torch.complex128, device="cuda")
    rc = lib.load().gwf_waveform_deriv(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid),
                                       dw.flags | lib.MIXED, off.data_ptr(), total, out.data_ptr(),
                                       None, None)
    assert rc == lib.GWF_E_UNSUPPORTED


def test_gps_scale_tc_against_oracle(lib, orc):
    """Coalescence times of order 1e9 s in the phase (the 2 pi f tc term
    reaches 1e13 rad): every derivative against the oracle with the phase
    scale of the tolerance including tc, and the Fisher matrix rebuilt from
    the derivatives unchanged by tc (it depends on |d h|^2 only)."""
    full = synth.bns1e4()
    wl = full.subset(np.arange(3)).with_npts(500)
    wl.tc_s = np.array([1.3e9, 1.0e9 + 0.37, 2.5e8])
    offsets, total = _offsets(wl.npts, 3)
    dh, st = _gpu(lib, wl, offsets, total)
    np.testing.assert_array_equal(st, 0)
    _check_against_oracle(orc, wl, dh, offsets, total)
    w0 = wl.subset(np.arange(wl.n))
    w0.tc_s = None
    dh0, _ = _gpu(lib, w0, offsets, total)
    F, F0 = _fisher_from(orc, wl, dh, offsets), _fisher_from(orc, w0, dh0, offsets)
    assert _fisher_close(F, F0) <= 1e-11

"""The C ABI library loads, exports every symbol include/gwf.h declares,
and rejects malformed arguments on the host before any launch (no GPU
needed: these calls never reach a kernel)."""
import ctypes
import os
import re

import pytest

from paper_2207_06910_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gwf.h")).read()
    return sorted(set(re.findall(r"\b(gwf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = _declared()
    assert {"gwf_snr", "gwf_fisher", "gwf_invert"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert lib.gwf_version() == 7


def test_network_interferometer_count():
    w = synth.bns1e4(n=2)
    assert binding.n_ifo(w.sites) == 5
    assert binding.n_ifo([synth.site("H1")]) == 1
    assert binding.n_ifo([synth.site("ETS"), synth.site("ETMR")]) == 6


def _descs(n=3):
    ev = binding.Events(n, n, 1, None)              # non-NULL dummy pointer, never dereferenced
    net, keep = binding.network([synth.site("H1")])
    grid = binding.Grid(0, 8, None, 16)
    return ev, net, grid, keep


def test_invalid_arguments_rejected_on_host():
    lib = binding.load()
    ev, net, grid, keep = _descs()
    B = ctypes.byref
    # missing outputs
    assert lib.gwf_fisher(B(ev), B(net), B(grid), 0, 0.0, None, None, None, None, None) == 1
    assert b"required" in lib.gwf_last_error()
    # n < 1, ld < n
    bad = binding.Events(0, 1, 1, None)
    assert lib.gwf_snr(B(bad), B(net), B(grid), 0, 8, None, None, None) == 1
    bad = binding.Events(4, 3, 1, None)
    assert lib.gwf_snr(B(bad), B(net), B(grid), 0, 8, None, None, None) == 1
    # unknown flag bit, unsupported grid kind
    assert lib.gwf_snr(B(ev), B(net), B(grid), 0x80, 8, None, None, None) == 1
    g2 = binding.Grid(7, 8, None, 16)
    assert lib.gwf_snr(B(ev), B(net), B(g2), 0, 8, None, None, None) == 2
    # bad network: too many sites, non-finite geometry, non-positive S0
    s = synth.site("H1")
    for sites in ([s] * 9, [synth.Site(float("nan"), 0, 0, 1, 0)], [synth.Site(0, 0, 0, 1, 0, 0.0)]):
        n2, k2 = binding.network(sites)
        assert lib.gwf_snr(B(ev), B(n2), B(grid), 0, 8, None, None, None) == 1
    # waveform: missing offsets or h, total < 1
    assert lib.gwf_waveform(B(ev), B(net), B(grid), 0, None, 10, 8, None, None) == 1
    assert lib.gwf_waveform(B(ev), B(net), B(grid), 0, 8, 10, None, None, None) == 1
    assert lib.gwf_waveform(B(ev), B(net), B(grid), 0, 8, 0, 8, None, None) == 1
    # per-interferometer Fisher: outputs required, no mixed form
    assert lib.gwf_fisher_ifo(B(ev), B(net), B(grid), 0, None, 8, None) == 1
    assert lib.gwf_fisher_ifo(B(ev), B(net), B(grid), 0, 8, None, None) == 1
    assert lib.gwf_fisher_ifo(B(ev), B(net), B(grid), binding.MIXED, 8, 8, None) == 2
    # strain derivatives: the same checks, and no mixed form
    assert lib.gwf_waveform_deriv(B(ev), B(net), B(grid), 0, None, 10, 8, None, None) == 1
    assert lib.gwf_waveform_deriv(B(ev), B(net), B(grid), 0, 8, 10, None, None, None) == 1
    assert lib.gwf_waveform_deriv(B(ev), B(net), B(grid), 0, 8, 0, 8, None, None) == 1
    assert lib.gwf_waveform_deriv(B(ev), B(net), B(grid), binding.MIXED, 8, 10, 8, None, None) == 2
    # inversion: P out of range, NaN threshold
    assert lib.gwf_invert(15, 3, 8, 1e50, None, 8, None, None, None, 8, None) == 1
    assert lib.gwf_invert(13, 3, 8, float("nan"), None, 8, None, None, None, 8, None) == 1
    # adjoint: missing outputs, non-finite weight, no mixed form
    assert lib.gwf_fisher_adjoint(B(ev), B(net), B(grid), 0, 8, None, 1.0, 1.0, None, 8, None) == 1
    assert lib.gwf_fisher_adjoint(B(ev), B(net), B(grid), 0, 8, None, float("inf"), 1.0, 8, 8, None) == 1
    assert lib.gwf_fisher_adjoint(B(ev), B(net), B(grid), 4, 8, None, 1.0, 1.0, 8, 8, None) == 2
    # explicit grids: offsets and frequencies required; the adjoint and plans refuse them
    gx = binding.Grid(binding.GRID_EXPLICIT, None, None, 16, None, 24)
    assert lib.gwf_snr(B(ev), B(net), B(gx), 0, 8, None, None, None) == 1
    gx = binding.Grid(binding.GRID_EXPLICIT, None, None, 16, 32, None)
    assert lib.gwf_fisher(B(ev), B(net), B(gx), 0, 0.0, 8, 8, None, 8, None) == 1
    gx = binding.Grid(binding.GRID_EXPLICIT, None, None, 16, 32, 24)
    assert lib.gwf_fisher_adjoint(B(ev), B(net), B(gx), 0, 8, None, 1.0, 1.0, 8, 8, None) == 2
    plan = ctypes.c_void_p()
    assert lib.gwf_plan_create(B(ev), B(net), B(gx), 0, None, B(plan), None) == 2
    assert len(lib.gwf_last_error()) > 0
    # plans invert by Cholesky, Cholesky with the SVD fallback or double-double Cholesky only
    for m in (2, 3, 7):
        opt = binding.PlanOptions(0, 1, 0, m)
        assert lib.gwf_plan_create(B(ev), B(net), B(grid), 0, B(opt), B(plan), None) == 1
        assert b"inv_method" in lib.gwf_last_error()
    # the static-workspace form: outputs, item length, grid bound, workspace size
    assert lib.gwf_fisher_static(B(ev), B(net), B(grid), 0, 4096, 100, None, 8, 8, None) == 1
    assert lib.gwf_fisher_static(B(ev), B(net), B(grid), 0, 100, 100, 8, 8, 8, None) == 1
    assert lib.gwf_fisher_static(B(ev), B(net), B(grid), 0, 4096, 1, 8, 8, 8, None) == 1
    big = binding.Events(10 ** 6, 10 ** 6, 1, None)
    assert lib.gwf_fisher_static(B(big), B(net), B(grid), 0, 4096, 20000, 8, 8, 8, None) == 1
    assert b"workspace" in lib.gwf_last_error()
    assert lib.gwf_fisher_static(B(ev), B(net), B(gx), 0, 4096, 100, 8, 8, 8, None) == 2
    # eccentricity needs the e0 array
    assert lib.gwf_snr(B(ev), B(net), B(grid), binding.ECCENTRIC, 8, None, None, None) == 1
    assert b"ecc" in lib.gwf_last_error()
    # an unknown noise-curve kind
    s = synth.site("H1")
    n3, k3 = binding.network([s])
    k3[0].psd_kind = 5
    assert lib.gwf_snr(B(ev), B(n3), B(grid), 0, 8, None, None, None) == 1


def test_covariance_options_rejected_on_host():
    """gwf_covariance: masks beyond P, fixed and marginalised overlapping,
    nothing left, negative or non-finite priors, priors beyond P, a sky level
    of 100% or more, theta or phi fixed or out of range, missing theta or sky
    output, unknown units, unknown method, SVD threshold outside [0, 1)."""
    lib = binding.load()
    B = ctypes.byref

    def opts(**kw):
        o = binding.CovOptions()
        o.cond_max = 1e50
        o.i_theta, o.i_phi = 3, 4
        for k, v in kw.items():
            if k == "prior":
                for i, x in v.items():
                    o.prior[i] = x
            else:
                setattr(o, k, v)
        return o

    def call(o, P=13, theta=8, sky=8):
        return lib.gwf_covariance(P, 3, 8, B(o), theta, None, 8, None, None, None, sky, None, None, 8, None)

    assert lib.gwf_covariance(13, 3, 8, None, None, None, 8, None, None, None, None, None, None, 8, None) == 1
    assert call(opts(fixed_mask=1 << 13)) == 1
    assert call(opts(marg_mask=1 << 11), P=11) == 1
    assert call(opts(fixed_mask=3, marg_mask=2)) == 1
    assert b"both" in lib.gwf_last_error()
    assert call(opts(fixed_mask=1, marg_mask=2), P=2) == 1
    assert call(opts(prior={5: -1.0})) == 1
    assert call(opts(prior={5: float("inf")})) == 1
    assert call(opts(prior={12: 1.0}), P=11) == 1
    assert call(opts(cond_max=float("nan"))) == 1
    assert call(opts(sky_level=100.0)) == 1
    assert call(opts(sky_level=90.0, fixed_mask=1 << 3)) == 1
    assert b"fixed" in lib.gwf_last_error()
    assert call(opts(sky_level=90.0, i_phi=3)) == 1
    assert call(opts(sky_level=90.0, i_theta=13)) == 1
    assert call(opts(sky_level=90.0), theta=None) == 1
    assert call(opts(sky_level=90.0), sky=None) == 1
    assert call(opts(sky_level=90.0, sky_units=2)) == 1
    assert call(opts(method=5)) == 1
    assert call(opts(method=2, svals_thresh=1.0)) == 1
    assert call(opts(method=3, svals_thresh=float("nan"))) == 1


def test_basis_arguments_rejected_on_host():
    """gwf_fisher_basis: P outside 11-14, the tidal basis without tides (P =
    11, or 12: no tides and e0), unknown basis bits, a descriptor for another
    number of events, missing output."""
    lib = binding.load()
    B = ctypes.byref
    ev = binding.Events(3, 3, 8, None)
    assert lib.gwf_fisher_basis(10, 3, 8, B(ev), 1, 8, None, None) == 1
    assert lib.gwf_fisher_basis(15, 3, 8, B(ev), 1, 8, None, None) == 1
    assert lib.gwf_fisher_basis(11, 3, 8, B(ev), 2, 8, None, None) == 1
    assert lib.gwf_fisher_basis(12, 3, 8, B(ev), 2, 8, None, None) == 1
    assert lib.gwf_fisher_basis(13, 3, 8, B(ev), 8, 8, None, None) == 1
    assert lib.gwf_fisher_basis(13, 4, 8, B(ev), 1, 8, None, None) == 1
    assert lib.gwf_fisher_basis(13, 3, 8, B(ev), 1, None, None, None) == 1
    assert b"required" in lib.gwf_last_error()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.GwfError):
        binding.load()

"""GPU parity of gwf_fisher_ifo (the Fisher matrix of each interferometer on
its own) against the oracle's per-interferometer matrices, and its sum over
the interferometers against gwf_fisher's network matrix.

Tolerance as for gwf_fisher: |dGamma_ab| <= 1e-9 sqrt(Gamma_aa Gamma_bb)
per interferometer against the oracle.  The network matrix sums the same
per-point terms with the triangle's closure identity (two effective
interferometers instead of three arms), so the sum of the per-interferometer
matrices must equal it to rounding, 1e-12 of sqrt(Gamma_aa Gamma_bb).
"""
import numpy as np
import pytest

from paper_2207_06910_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2207_06910_amd import binding
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    binding.load()
    return binding


def _norm_err(F, R):
    """max |F - R| / sqrt(R_aa R_bb) over entries with nonzero diagonals;
    entries of zero rows must be zero in F."""
    d = np.sqrt(np.abs(np.einsum("...iie->...ie", R)))
    z = d == 0
    d = np.where(z, 1.0, d)
    e = np.abs(F - R) / (d[..., :, None, :] * d[..., None, :, :])
    zero = z[..., :, None, :] | z[..., None, :, :]
    assert np.all(F[zero] == 0)
    return np.where(zero, 0.0, e).max()


@pytest.mark.parametrize("case", ["bns", "mixed_duty"])
def test_fisher_ifo_against_oracle_and_network(lib, orc, case):
    """The triangle + two L network (BNS, tides, rotation) and the five-L
    mixed workload with each kind's parameter set and a 60% duty factor:
    every interferometer's matrix against the oracle's, zero where the
    interferometer is off or the row is outside the event's set, and the sum
    over interferometers against the network matrix."""
    if case == "bns":
        wl = synth.bns1e4().subset(np.arange(4)).with_npts(900)
    else:
        full = synth.mixed1e4(n=200)
        kind = full.meta["kind"]
        idx = np.r_[np.flatnonzero(kind == 0)[:3], np.flatnonzero(kind == 1)[:3]]
        wl = full.subset(idx).with_npts(700).with_duty_factor(0.6, seed=5)
    dw = lib.DeviceWorkload(wl)
    r = lib.fisher_ifo(dw)
    net = lib.fisher(dw)
    torch.cuda.synchronize()
    Fi = r["fisher_ifo"].cpu().numpy()
    np.testing.assert_array_equal(r["status"].cpu().numpy(), 0)
    ref = orc.fisher(wl, per_ifo=True)
    Ri = ref["fisher_ifo"]
    if wl.par_mask is not None:
        for d in range(Ri.shape[0]):
            orc.restrict_rows(Ri[d], wl.par_mask)
    if wl.active is not None:
        off = ~wl.active.astype(bool)
        assert off.any()
        assert np.all(Fi.transpose(0, 3, 1, 2)[off] == 0)
    assert _norm_err(Fi, Ri) <= 1e-9
    G = net["fisher"].cpu().numpy()
    assert _norm_err(Fi.sum(axis=0), G) <= 1e-12


def test_fisher_ifo_single_detector_equals_network(lib, orc):
    """One L detector without rotation (11 parameters): its only matrix is
    the network matrix itself, bit for bit (the same kernel with the same
    single interferometer), and matches the oracle."""
    wl = synth.bbh100().subset(np.arange(6))
    dw = lib.DeviceWorkload(wl)
    Fi = lib.fisher_ifo(dw)["fisher_ifo"].cpu().numpy()
    G = lib.fisher(dw)["fisher"].cpu().numpy()
    assert Fi.shape == (1, 11, 11, 6)
    assert np.array_equal(Fi[0], G)
    assert _norm_err(Fi, orc.fisher(wl, per_ifo=True)["fisher_ifo"]) <= 1e-9

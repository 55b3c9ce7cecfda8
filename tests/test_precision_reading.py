"""CPU: why the mixed form confines FP32 to the positive per-point noise
weight (sec. 4.1 on the conditioning of Fisher matrices; the FP32 plan of
the mixed form), on oracle Fisher matrices of BNS events of the benchmark
catalogue (13 parameters, kappa 1e10-3e11), inverted in 50-digit arithmetic.

(1) Per-point weights with relative errors up to e: the matrix is a sum of
    positive semidefinite terms w_k Re(d_k d_k^H), so perturbing each w_k by
    (1 + delta_k), |delta_k| <= e, gives (1 - e) Gamma <= Gamma' <= (1 + e)
    Gamma in the Loewner order and every sigma_i stays within
    [(1 + e)^-1/2, (1 - e)^-1/2] of its value, whatever kappa is.
(2) Errors of FP32 size (1e-7 of sqrt(Gamma_ii Gamma_jj)) in the elements
    themselves, which FP32 derivative products or FP32 sums would leave:
    sigma moves by tens of percent or the matrix stops being positive
    definite, on every event.

Both use the two L-shaped sites of the catalogue's network (one
interferometer each), the oracle's strain derivatives on the events' grids
and its noise weights 4 w / S_n; the assembled matrices equal the oracle's
Fisher matrices to 1e-14 of sqrt(Gamma_ii Gamma_jj)."""
import numpy as np
import pytest

from paper_2207_06910_amd import synth


@pytest.fixture(scope="module")
def case(orc):
    wl = synth.bns1e4(n=200).subset(np.arange(0, 200, 25))
    wl.sites = wl.sites[1:]                          # the two L sites: interferometer d is site d
    assert orc.n_ifo(wl.site_array()) == len(wl.sites)
    F = orc.fisher(wl)["fisher"]
    ref = orc.covariance(F, dps=50, method="cho_svd")
    offs = np.concatenate([[0], np.cumsum(wl.npts)[:-1]]).astype(np.int64)
    dh = orc.waveform_derivs(wl, offs, int(wl.npts.sum()))
    terms = []                                       # per event: [(derivatives [P][k], weights [k]) per site]
    for e in range(wl.n):
        f, w = orc.grid(wl.fmin[e], orc.cut_frequency(wl.par[0, e], wl.par[1, e]), int(wl.npts[e]))
        sl = slice(offs[e], offs[e] + wl.npts[e])
        terms.append([(dh[:, d, sl], orc.noise_weight(s, f, w)) for d, s in enumerate(wl.sites)])
    return wl, F, ref, terms


def _assemble(terms, P, scale=None, rng=None, e=0.0):
    G = np.zeros((P, P, len(terms)))
    for ev, per_site in enumerate(terms):
        for D, nw in per_site:
            if e:
                nw = nw * (1.0 + rng.uniform(-e, e, nw.shape))
            G[:, :, ev] += np.real((D * nw) @ D.conj().T)
    return G


def _norm(F):
    d = np.sqrt(np.einsum("iie->ie", F))
    return d[:, None, :] * d[None, :, :]


def test_assembly_matches_oracle_fisher(case):
    wl, F, ref, terms = case
    G = _assemble(terms, F.shape[0])
    assert (np.abs(G - F) / _norm(F)).max() < 1e-14
    assert np.all(ref["status"] == 0) and ref["cond"].min() > 1e10


@pytest.mark.parametrize("e", [1e-2, 1e-3])
def test_weight_errors_bounded_at_any_kappa(case, orc, e):
    """The perturbed matrices are summed in FP64, whose own rounding moves
    sigma by about kappa u (7e-6 at kappa 1e11, seen with e = 1e-7); the
    check allows 4 kappa u beyond the Loewner bound, so it is meaningful for
    e well above that floor."""
    wl, F, ref, terms = case
    Gp = _assemble(terms, F.shape[0], rng=np.random.default_rng(11), e=e)
    got = orc.covariance(Gp, dps=50, method="cho_svd")
    assert np.all(got["status"] == 0)
    r = got["sigma"] / ref["sigma"]
    floor = 4 * ref["cond"] * 2.0 ** -53
    assert np.all(floor < 0.25 * e)
    assert np.all(r >= (1 + e) ** -0.5 - floor) and np.all(r <= (1 - e) ** -0.5 + floor), np.abs(r - 1).max()
    # the bound is reached in order of magnitude: the weights' errors are not averaged away
    assert np.abs(r - 1).max() > 0.01 * e


def test_element_errors_of_fp32_size_lose_sigma(case, orc):
    wl, F, ref, terms = case
    eps = np.random.default_rng(12).normal(size=F.shape) * 1e-7
    eps = 0.5 * (eps + eps.transpose(1, 0, 2))
    got = orc.covariance(F + eps * _norm(F), dps=50, method="cho_svd")
    with np.errstate(invalid="ignore"):
        rel = np.abs(got["sigma"] / ref["sigma"] - 1)
    worst = np.where(np.isnan(rel).any(axis=0), np.inf, np.nanmax(rel, axis=0))
    # every event is off by more than 10% (or no longer positive definite)
    assert np.all(worst > 0.1), worst

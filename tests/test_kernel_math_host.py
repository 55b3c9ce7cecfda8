"""The kernels' per-point mathematics (gwf_model.hpp, compiled for the host
by tests/model_host) against the oracle, on the CPU.  This checks the
analytic derivatives, the closed-form antenna patterns, the triangle
reduction and the Gram structure without a GPU; the parity claims of the
library itself rest on the GPU tests."""
import numpy as np
import pytest

import model_host
from paper_2207_06910_amd import synth


def _err(a, b):
    d = np.sqrt(np.einsum("iie->ie", b["fisher"]))
    return np.abs(a["fisher"] - b["fisher"]) / (d[:, None, :] * d[None, :, :])


@pytest.mark.parametrize("flags", [0, synth.FLAG_EARTH_ROT, synth.FLAG_TIDAL,
                                   synth.FLAG_TIDAL | synth.FLAG_EARTH_ROT])
def test_host_model_matches_oracle(orc, flags):
    wl = synth.bns1e4(n=5).with_npts(1500)
    wl.flags = flags
    a = model_host.fisher(wl)
    b = orc.fisher(wl)
    assert np.all(a["status"] == 0)
    np.testing.assert_allclose(a["snr"], b["snr"], rtol=1e-13)
    assert _err(a, b).max() < 1e-12


def test_host_model_bbh_single_detector(orc):
    wl = synth.bbh100(n=6)
    a = model_host.fisher(wl)
    b = orc.fisher(wl)
    np.testing.assert_allclose(a["snr"], b["snr"], rtol=1e-13)
    assert _err(a, b).max() < 1e-12


def test_host_model_invalid_events_flagged():
    wl = synth.bbh100(n=4)
    wl.par[1, 0] = 0.3          # eta > 1/4
    wl.par[2, 1] = -1.0         # dL < 0
    wl.par[3, 2] = np.nan       # theta
    a = model_host.fisher(wl)
    assert a["status"][0] == 1 and a["status"][1] == 1 and a["status"][2] == 8 and a["status"][3] == 0


def test_host_model_mixed_weight_bound(orc):
    """Mixed form on the host: only the noise weight is FP32, so SNR^2 and
    every Fisher element move by at most eps (relative to sqrt(G_ii G_jj)),
    eps the weight's relative error; here eps = 3e-7 covers the FP32
    exponential of an argument in [-1/2, 1/2] and a few FP32 roundings."""
    wl = synth.bns1e4(n=5).with_npts(1500)
    a = model_host.fisher(wl, flags=wl.flags | 4)
    b = model_host.fisher(wl)
    assert np.all(a["status"] == 0)
    np.testing.assert_allclose(a["snr"] ** 2, b["snr"] ** 2, rtol=3e-7)
    e = _err(a, b).max()
    assert 0 < e < 3e-7, e

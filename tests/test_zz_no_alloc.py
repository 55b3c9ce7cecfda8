"""GPU: gwf_fisher_static, the batched form with its workspace in the
library's fixed device array (no device allocation), against the plan
(gwf_plan_fisher) with the same item length: the same kernels over the same
work items, so the Fisher matrices, SNRs and statuses must agree bit for
bit.  Two calls in a row, the second on a smaller catalogue, so that the
second call finds the first one's contents in the array; the first one is
also checked against the oracle on sampled events (SNR 1e-12, Fisher 1e-9
of sqrt(G_ii G_jj))."""
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


def _np(r):
    return {k: v.cpu().numpy() for k, v in r.items()}


def _plan(lib, dw, chunk, mixed=False):
    plan = lib.Plan(dw, chunk=chunk, mixed=mixed)
    r = plan.run()
    torch.cuda.synchronize()
    out = _np(r)
    plan.close()
    return out


def test_static_workspace_matches_plan_twice(lib, orc):
    full = synth.bns1e4()
    big = full.subset(np.arange(1500))            # grids of 2000-20000 points
    small = full.subset(np.arange(1500, 1620)).with_npts(700)
    small.npts[::7] = 5000                         # ragged: one or two items per event
    chunk = 4096
    for wl, label in ((big, "first call, 1500 events"), (small, "second call, 120 events")):
        dw = lib.DeviceWorkload(wl)
        g = _np(lib.fisher_static(dw, chunk=chunk))
        torch.cuda.synchronize()
        ref = _plan(lib, dw, chunk)
        assert np.all(g["status"] == 0), label
        for k in ("fisher", "snr", "status"):
            assert np.array_equal(g[k], ref[k]), (label, k)
        if wl is big:
            idx = np.random.default_rng(9).choice(wl.n, 5, replace=False)
            o = orc.fisher(wl.subset(idx))
            assert np.max(np.abs(g["snr"][idx] / o["snr"] - 1)) <= 1e-12
            d = np.sqrt(np.einsum("iie->ie", o["fisher"]))
            err = np.abs(g["fisher"][:, :, idx] - o["fisher"]) / (d[:, None, :] * d[None, :, :])
            assert err.max() <= 1e-9, err.max()
        print(f"{label}: equal to the plan bit for bit")


def test_static_mixed_and_non_tidal_and_flags(lib):
    """The mixed form, a catalogue without tides on one L site without
    rotation, and an event whose grid exceeds npts_max (flagged invalid,
    zero Fisher), each against the plan."""
    wl = synth.bns1e4(n=64).with_npts(3000)
    dw = lib.DeviceWorkload(wl)
    g = _np(lib.fisher_static(dw, chunk=1024, mixed=True))
    ref = _plan(lib, dw, 1024, mixed=True)
    for k in ("fisher", "snr", "status"):
        assert np.array_equal(g[k], ref[k]), ("mixed", k)
    wl2 = synth.bbh100(n=40)
    dw2 = lib.DeviceWorkload(wl2)
    g = _np(lib.fisher_static(dw2, chunk=512))
    ref = _plan(lib, dw2, 512)
    for k in ("fisher", "snr", "status"):
        assert np.array_equal(g[k], ref[k]), ("bbh", k)
    wl3 = synth.bns1e4(n=8).with_npts(900)
    wl3.npts[3] = 2000
    dw3 = lib.DeviceWorkload(wl3)
    g = _np(lib.fisher_static(dw3, chunk=512, npts_max=1000))
    assert g["status"][3] == 1 and np.all(g["fisher"][:, :, 3] == 0)
    keep = np.array([e for e in range(8) if e != 3])
    ref = _plan(lib, lib.DeviceWorkload(wl3.subset(keep)), 512)
    assert np.array_equal(g["fisher"][:, :, keep], ref["fisher"])


def test_static_rejects_a_catalogue_beyond_its_workspace(lib):
    """10^5 events with grids up to 20000 points in items of 256 points
    need far more than the fixed array: refused on the host, nothing
    launched."""
    wl = synth.bns1e4(n=2)
    dw = lib.DeviceWorkload(wl)
    with pytest.raises(lib.GwfError, match="workspace"):
        lib.fisher_static(dw, chunk=256, npts_max=1 << 29)

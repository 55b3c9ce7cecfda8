"""GPU: the batched form (gwf_plan_*, work items + HIP graph)
against the plain kernel and the oracle.  The two forms sum the same
per-point terms in a different order, so they agree to rounding (<= 1e-13
relative on SNR, <= 1e-12 normalised on Fisher elements)."""
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


def _ferr(F, R):
    d = np.sqrt(np.abs(np.einsum("iie->ie", R)))
    return (np.abs(F - R) / (d[:, None, :] * d[None, :, :])).max()


@pytest.mark.parametrize("chunk,use_graph", [(512, True), (2048, False), (0, True)])
def test_plan_matches_plain_and_oracle(lib, orc, chunk, use_graph):
    full = synth.bns1e4()
    wl = full.subset(np.r_[np.argmin(full.npts), np.argmax(full.npts), np.arange(40)])
    dw = lib.DeviceWorkload(wl)
    plain = _np(lib.fisher(dw))
    plan = lib.Plan(dw, chunk=chunk, use_graph=use_graph)
    info = plan.info()
    assert info["n_items"] >= wl.n and (chunk == 0 or info["chunk"] == chunk)
    b = _np(plan.run())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(b["status"], 0)
    np.testing.assert_allclose(b["snr"], plain["snr"], rtol=1e-13)
    assert _ferr(b["fisher"], plain["fisher"]) <= 1e-12
    ref = orc.fisher(wl.subset(np.arange(6)))
    np.testing.assert_allclose(b["snr"][:6], ref["snr"], rtol=1e-12)
    assert _ferr(b["fisher"][:, :, :6], ref["fisher"]) <= 1e-9
    plan.close()


def test_graph_replays_with_eager_work_between(lib):
    """Replay the captured graph several times, with unrelated eager work
    and synchronisations in between; every replay equals the first."""
    wl = synth.bns1e4(n=64)
    dw = lib.DeviceWorkload(wl)
    plan = lib.Plan(dw, chunk=1024)
    out = plan.run(invert=True)
    torch.cuda.synchronize()
    first = _np(out)
    for i in range(4):
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (x * x).sum().item()
        plan.run(invert=True, out=out)
        torch.cuda.synchronize()
        r = _np(out)
        for k in ("fisher", "snr", "status", "sigma", "cond"):
            assert np.array_equal(r[k], first[k], equal_nan=True), k
    # the inversion inside the graph equals gwf_invert on the same Fisher
    inv = _np(lib.invert(out["fisher"], torch.zeros_like(out["status"])))
    assert np.array_equal(inv["sigma"], first["sigma"], equal_nan=True)
    plan.close()


def test_plan_follows_parameter_updates_and_rejects_grid_changes(lib):
    wl = synth.bns1e4(n=20)
    dw = lib.DeviceWorkload(wl)
    plan = lib.Plan(dw, chunk=2048)
    a = _np(plan.run())
    dw.par[2] *= 2.0                       # distances doubled in place
    b = _np(plan.run())
    np.testing.assert_allclose(b["snr"], a["snr"] / 2, rtol=1e-14)
    dw.npts[3] += 1                        # grid length changed after plan creation
    c = _np(plan.run())
    torch.cuda.synchronize()
    assert c["status"][3] == 1 and np.all(np.delete(c["status"], 3) == 0)
    plan.close()


# ----------------------------------------------------------- mixed form
EPS_W = 1e-6   # relative error of the FP32 noise weight: FP32 exponential of an
               # argument in [-1/2, 1/2] (a few ulp on the device) and about five
               # FP32 roundings, ~5e-7, with a factor of two to spare


def test_mixed_plan_bounds(lib, orc):
    """Mixed form (FP32 noise weight, everything else FP64).  A per-point
    weight error |e_k| <= EPS_W keeps (1 - EPS_W) G <= G' <= (1 + EPS_W) G,
    hence SNR within EPS_W/2 and |G'_ij - G_ij| <= EPS_W sqrt(G_ii G_jj)
    (Cauchy-Schwarz), both checked against the oracle; sigma_i (mpmath
    inversion of the GPU matrices) within 1e-3 of the oracle's on every event
    whose condition number is below 1e13, where FP64 rounding in the sums
    moves sigma by less than that."""
    full = synth.bns1e4()
    idx = np.unique(np.r_[np.argmin(full.npts), np.argmax(full.npts),
                          np.random.default_rng(21).choice(full.n, 14, replace=False)])
    wl = full.subset(idx)
    dw = lib.DeviceWorkload(wl)
    pm = lib.Plan(dw, chunk=2048, mixed=True)
    m = _np(pm.run(invert=True))
    pm.close()
    torch.cuda.synchronize()
    assert np.all(m["status"] & 1 == 0)
    ref = orc.fisher(wl)
    np.testing.assert_allclose(m["snr"], ref["snr"], rtol=EPS_W / 2 + 1e-12)
    e = _ferr(m["fisher"], ref["fisher"])
    assert e <= EPS_W + 1e-9, e
    inv = orc.covariance(ref["fisher"], dps=40)
    invm = orc.covariance(m["fisher"], dps=40)
    ok = inv["cond"] < 1e13
    assert ok.sum() >= 5
    rel = np.abs(invm["sigma"][:, ok] / inv["sigma"][:, ok] - 1)
    assert rel.max() <= 1e-3, rel.max()
    print(f"mixed: SNR {np.abs(m['snr'] / ref['snr'] - 1).max():.1e}, Fisher {e:.1e}, "
          f"sigma (kappa < 1e13, {ok.sum()} events) {rel.max():.1e}")


def test_mixed_waveform(lib, orc):
    """Mixed strain: FP32 amplitude (exponential of a reduced argument) and
    FP32 sin/cos of the FP64-reduced phases, each accurate to ~1e-7, so the
    strain stays within 1e-6 of the FP64 kernel's, relative to the point's
    largest |h| over interferometers."""
    wl = synth.bns1e4(n=6)
    dw = lib.DeviceWorkload(wl)
    h = lib.waveform(dw)["h"].cpu().numpy()
    hm = lib.waveform(dw, mixed=True)["h"].cpu().numpy()
    scale = np.abs(h).max(axis=0)
    err = (np.abs(hm - h) / scale[None, :]).max()
    assert err <= 1e-6, err


def test_catalogue_1e6_plan(lib, orc):
    """The 10^6-event BBH/BNS/NSBH catalogue (more than 2^31 grid points in
    total; each kind with its own parameter set) in one launch
    with inversion: every event's Fisher is
    computed, the identity Gamma_dLdL dL^2 = SNR^2 holds for all of them,
    sampled events of each kind match the oracle, and ill-conditioned or
    non-positive-definite matrices are flagged, never silently inverted."""
    wl = synth.catalog1e6()
    assert int(wl.npts.sum()) > 2 ** 31
    dw = lib.DeviceWorkload(wl)
    plan = lib.Plan(dw, chunk=8192)
    out = plan.run(invert=True)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    snr = out["snr"].cpu().numpy()
    assert np.all(st & 1 == 0) and np.all(st & 8 == 0)
    F_dl = out["fisher"][2, 2].cpu().numpy()
    np.testing.assert_allclose(F_dl * wl.par[2] ** 2, snr ** 2, rtol=1e-12)
    sig = out["sigma"].cpu().numpy()
    # each kind's own rows: 11 for BBH, 13 for BNS, 12 for NSBH
    inn = ((wl.par_mask[None, :].astype(np.int64) >> np.arange(13)[:, None]) & 1).astype(bool)
    assert np.array_equal(inn.sum(axis=0), np.choose(wl.meta["kind"], [11, 13, 12]))
    assert np.all(np.isfinite(sig[:, st == 0][inn[:, st == 0]]))
    assert np.all(np.isnan(sig[:, st == 0][~inn[:, st == 0]])) and np.all(np.isnan(sig[:, st != 0]))
    kind = wl.meta["kind"]
    idx = np.r_[[np.flatnonzero(kind == k)[0] for k in range(3)]]
    ref = orc.fisher(wl.subset(idx))
    F = out["fisher"][:, :, torch.as_tensor(idx, device="cuda")].cpu().numpy()
    np.testing.assert_allclose(snr[idx], ref["snr"], rtol=1e-12)
    both = inn[:, None, idx] & inn[None, :, idx]
    assert np.all(F[~both] == 0) and np.all(ref["fisher"][~both] == 0)
    d = np.sqrt(np.where(inn[:, idx], np.einsum("iie->ie", ref["fisher"]), 1.0))
    assert (np.abs(F - ref["fisher"]) / (d[:, None, :] * d[None, :, :])).max() <= 1e-9
    plan.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_full_catalogue_in_the_bench_launch(lib, orc, mixed):
    """Both batched forms on the whole 10^4-event BNS catalogue in the
    benchmark's launch (16384-point items, four workgroups per compute unit,
    HIP graph, inversion): every event valid and inverted or flagged, the
    identity Gamma_dLdL dL^2 = SNR^2 for all of them (both sides carry the
    same weights, so it holds to rounding in either form), and sampled
    events against the oracle at the form's bar (FP64: SNR 1e-12, Fisher
    1e-9; mixed: the weight-error bounds of test_mixed_plan_bounds)."""
    full = synth.bns1e4()
    dw = lib.DeviceWorkload(full)
    plan = lib.Plan(dw, chunk=16384, mixed=mixed)
    g = _np(plan.run(invert=True))
    plan.close()
    torch.cuda.synchronize()
    st = g["status"]
    assert np.all(st & 1 == 0) and np.all(st & 8 == 0)
    assert (st == 0).sum() >= 0.99 * full.n
    np.testing.assert_allclose(g["fisher"][2, 2] * full.par[2] ** 2, g["snr"] ** 2, rtol=1e-12)
    idx = np.random.default_rng(5 + mixed).choice(full.n, 8, replace=False)
    ref = orc.fisher(full.subset(idx))
    tol_s, tol_f = (EPS_W / 2 + 1e-12, EPS_W + 1e-9) if mixed else (1e-12, 1e-9)
    np.testing.assert_allclose(g["snr"][idx], ref["snr"], rtol=tol_s)
    assert _ferr(g["fisher"][:, :, idx], ref["fisher"]) <= tol_f

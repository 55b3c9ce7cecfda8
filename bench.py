"""Benchmark of the Fisher/SNR hot path on one MI355X.

One step = the whole path over the 10^4-event BNS catalogue: SNR and Fisher
matrices (gwf_fisher, one fused kernel) followed by the batched FP64
inversion (gwf_invert), with every input already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-sample M]

Prints one JSON line: throughput in events/s, the roofline of the dominant
kernel (Fisher) measured with HIP events on its stream, and the CPU oracle
timed on a bounded sample of the same catalogue.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 vector peak
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E

# HBM bytes per launch of each kernel on the BNS catalogue, from the
# FETCH_SIZE and WRITE_SIZE counter passes summarised in
# profiles/bns1e4_hbm_counters.md (calibrated against a 256 MiB copy: fetch
# x 2.000, write x 1.000).  Set an entry to None when its kernel changes.
MEASURED_TRAFFIC = {
    "items_kernel<tidal,rot>": 63.58e6,
    "items_kernel<tidal,rot,mixed>": 65.59e6,
    "fisher_kernel<tidal,rot>": 68.57e6,
    "waveform_kernel<rot,tidal>": 7853.20e6,
    "waveform_kernel<rot,tidal,mixed>": 7880.95e6,
    "waveform_deriv_kernel<rot,tidal>": 10305.77e6,
}

# VALU instructions (wavefront instructions, SQ_INSTS_VALU, MFMA included) per
# launch of the Fisher kernels on the BNS catalogue, from the counter pass
# summarised in profiles/bns1e4_flop_counters.md.  A wave64 VALU instruction
# occupies its SIMD for 4 cycles, so the VALU busy fraction at the nominal
# clock is 4 x SQ_INSTS_VALU / (1024 SIMDs x 2.4 GHz x kernel time).  Set an
# entry to None when its kernel changes.
MEASURED_VALU_INSTS = {
    "items_kernel<tidal,rot>": 1.2594e9,
    "items_kernel<tidal,rot,mixed>": 1.2592e9,
    "fisher_kernel<tidal,rot>": 1.3111e9,
}
N_SIMD, CLOCK_HZ = 1024, 2.4e9


def valu_busy(kernel: str, kernel_ms: float):
    n = MEASURED_VALU_INSTS.get(kernel)
    return None if n is None else round(4.0 * n / (N_SIMD * CLOCK_HZ * kernel_ms * 1e-3), 4)


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# FP64 flops per grid point executed by the kernels, counted from their
# gfx950 instruction stream in this build (v_fma/v_fmac = 2, v_mul/v_add = 1,
# the MFMA as its 512 flops per four-block 4x4x4 instruction) for the
# instantiation the benchmarks run: tides, Earth rotation, analytic PSDs.
# Split by where the work sits: once per point, per site, per effective
# interferometer (n_eff = 1 per L site, 2 per closed triangle).
#   items_kernel (FP64)   point 223 (grid, amplitude, PN series, sidereal
#                         sin/cos, phase-only coefficients, staging),
#                         site 57 (hour angle, root of the PSD weight and the
#                         weighted trigonometric basis, arrival-time
#                         derivatives), interferometer 213 (six pattern
#                         polynomials, derivative vectors, 5x5 rank-2 update,
#                         moments); MFMA 128 (16 per 64 points)
#   items_kernel (mixed)  the same with the PSD's rational part in FP32:
#                         site 35 FP64 (+ 14 FP32)
#   adjoint_items_kernel  point 412 (the point set-up and the Gbar inner
#                         products of the point's vectors), site 115, interferometer 294
#                         (two points per lane and iteration; points past an item's
#                         end run at zero weight and are not in the model)
# The counter passes (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes and
# SQ_INSTS_VALU_MFMA_MOPS_F64 x 512) confirm these per launch.
KERNEL_FLOPS = {
    "items": {"point": 223, "site": 57, "ifo": 213, "mfma": 128},
    "items_mixed": {"point": 223, "site": 35, "ifo": 213, "mfma": 128},
    "adjoint": {"point": 412, "site": 115, "ifo": 294, "mfma": 0},
}
# A dense per-(point, interferometer) count (Gram 2P(P+1), weighting 2P,
# SNR 4, derivative assembly 8P, projection 120, PN 200 per point): the work
# of evaluating every interferometer's full P x P Gram, which the kernels'
# exact identities avoid
DENSE_PER_POINT_IFO = lambda P: 2 * P * (P + 1) + 2 * P + 4 + 8 * P + 120


def kernel_flops(wl, kind: str) -> dict:
    """Executed FP64 flops per launch of a kernel on workload wl (KERNEL_FLOPS)."""
    k = KERNEL_FLOPS[kind]
    n_site = len(wl.sites)
    n_eff = sum(2 if s.shape == 1 else 1 for s in wl.sites)
    pts = float(np.sum(wl.npts, dtype=np.int64))
    valu = (k["point"] + k["site"] * n_site + k["ifo"] * n_eff) * pts
    mfma = k["mfma"] * pts
    n_ifo = sum(3 if s.shape == 1 else 1 for s in wl.sites)
    dense = (DENSE_PER_POINT_IFO(wl.npar) * n_ifo + 200) * pts
    return {"valu": valu, "mfma": mfma, "total": valu + mfma, "dense": dense,
            "per_point": k["point"] + k["site"] * n_site + k["ifo"] * n_eff + k["mfma"]}


def cpu_baseline(wl, sample: int):
    """The oracle, as it stands, on a seeded sample of the catalogue:
    C++ SNR + Fisher (OpenMP) and the mpmath inversion.  Returns the
    baseline record and the oracle's results with the sampled indices."""
    import oracle
    threads = min(len(os.sched_getaffinity(0)), 16)
    idx = np.sort(np.random.default_rng(2207069101).choice(wl.n, sample, replace=False))
    sub = wl.subset(idx)
    oracle.load()
    t0 = time.perf_counter()
    r = oracle.fisher(sub, nthreads=threads)
    t1 = time.perf_counter()
    inv = oracle.covariance(r["fisher"], dps=30, method="cho_svd")
    t2 = time.perf_counter()
    rec = {"value": sample / (t2 - t0), "unit": "events/s", "cores": threads, "kind": "oracle",
           "sample": f"{sample} seeded events of the same catalogue ({int(sub.npts.sum())} grid "
                     f"points); Fisher+SNR {t1 - t0:.2f} s on {threads} threads, mpmath "
                     f"inversion (Cholesky, SVD where it fails) {t2 - t1:.2f} s"}
    rec["cpu_model"] = cpu_model()
    # not timed: the well-conditioned 9-parameter block of the same matrices
    keep = [k for k in range(r["fisher"].shape[0]) if k not in BLOCK_FIXED]
    F9 = np.ascontiguousarray(r["fisher"][np.ix_(keep, keep)])
    inv9 = oracle.covariance(F9, dps=30)
    return rec, {"idx": idx, "snr": r["snr"], "fisher": r["fisher"], "sigma": inv["sigma"],
                 "cond": inv["cond"], "sigma9": inv9["sigma"], "cond9": inv9["cond"]}


U64 = 2.0 ** -53
# the 9-parameter block of the well-conditioned comparison: spins and
# deformabilities held fixed (rows chi1z, chi2z, Lambda1, Lambda2 removed)
BLOCK_FIXED = (9, 10, 11, 12)
KAPPA_WELL = 1e5            # sigma parity <= 1e-9 asserted at or below this kappa
KAPPA_MIXED = 1e12          # the mixed form's sigma bar applies below this kappa


def _round(x, d=3):
    return None if x is None or not np.isfinite(x) else float(f"{x:.{d}g}")


def error_report(res, ref) -> dict:
    """Errors of one form's outputs against the oracle on the sampled events.

    SNR relative error; Fisher elements normalised by sqrt(G_ii G_jj), as the
    maximum and per element (upper triangle, row-major); sigma_i relative
    error of the full matrices per parameter and per decade of the condition
    number kappa, with the events whose sigma is NaN on the GPU but finite in
    the oracle counted apart (never skipped); the first-order bound
    |dsigma_i/sigma_i| <= (P/2) kappa eps_e + 1e3 kappa u per event, eps_e the
    event's largest normalised Fisher error (dC = -C dGamma C, with
    lambda_min of the unit-diagonal matrix >= 1/kappa); and the sigmas of the
    9-parameter block with spins and deformabilities fixed (kappa 1e3-1e8),
    where the Fisher error alone decides the sigma error."""
    i = ref["idx"]
    P = ref["fisher"].shape[0]
    snr = np.abs(res["snr"][i] / ref["snr"] - 1)
    F = res["fisher"][:, :, i]
    d = np.sqrt(np.abs(np.einsum("iie->ie", ref["fisher"])))
    ferr = np.abs(F - ref["fisher"]) / (d[:, None, :] * d[None, :, :])
    eps = ferr.max(axis=(0, 1))
    sg_g, sg_r = res["sigma"][:, i], ref["sigma"]
    both = np.isfinite(sg_g) & np.isfinite(sg_r)
    # a NaN sigma counts against the form wherever the GPU matrix is provably
    # positive definite: P kappa eps < 1 (Weyl: the normalised matrix's
    # smallest eigenvalue, at least 1/kappa, moves by at most P eps)
    provable = P * ref["cond"] * eps < 1.0
    nan_gpu = np.isfinite(sg_r) & ~np.isfinite(sg_g) & provable[None, :]
    nan_unprovable = int((np.isfinite(sg_r) & ~np.isfinite(sg_g) & ~provable[None, :]).any(axis=0).sum())
    sg = np.where(both, np.abs(sg_g / np.where(both, sg_r, 1.0) - 1), np.nan)
    kap = ref["cond"]
    ev_err = np.nanmax(np.where(both, sg, -1.0), axis=0)       # per event, -1 if none
    bound = 0.5 * P * kap * eps + 1e3 * kap * U64
    in_bound = (ev_err <= bound) & ~nan_gpu.any(axis=0)
    decades = []
    for lo in range(9, 17):
        m = (kap >= 10.0 ** lo) & (kap < 10.0 ** (lo + 1))
        if not m.any():
            continue
        e = ev_err[m]
        decades.append({"kappa": f"1e{lo}-1e{lo + 1}", "events": int(m.sum()),
                        "max_rel": _round(float(e.max())), "median_rel": _round(float(np.median(e))),
                        "nan_events": int(nan_gpu[:, m].any(axis=0).sum())})
    mixed_sel = kap < KAPPA_MIXED
    sub = ev_err[mixed_sel]
    iu = np.triu_indices(P)
    out = {"snr_max_rel": float(snr.max()), "fisher_max_norm": float(ferr.max()),
           "fisher_max_norm_per_element_upper": [_round(float(x), 2) for x in ferr.max(axis=2)[iu]],
           "sigma_max_rel_per_param": [_round(float(np.nanmax(sg[k]))) for k in range(P)],
           "sigma_by_kappa": decades,
           "sigma_nan_events": int(nan_gpu.any(axis=0).sum()),
           "sigma_nan_events_not_provably_pd": nan_unprovable,
           "sigma_within_first_order_bound": float(np.mean(in_bound)),
           f"sigma_max_rel_kappa_lt_{KAPPA_MIXED:.0e}": _round(float(sub.max())) if sub.size else None,
           f"sigma_nan_kappa_lt_{KAPPA_MIXED:.0e}": int(nan_gpu[:, mixed_sel].any(axis=0).sum()),
           f"events_kappa_lt_{KAPPA_MIXED:.0e}": int(mixed_sel.sum()),
           "events": int(len(i))}
    if "sigma9" in res and "sigma9" in ref:
        s9g, s9r, k9 = res["sigma9"][:, i], ref["sigma9"], ref["cond9"]
        e9 = np.abs(s9g / s9r - 1).max(axis=0)
        e9 = np.where(np.isfinite(e9), e9, np.inf)
        well = k9 <= KAPPA_WELL
        out["block9"] = {"fixed": "chi1z, chi2z, Lambda1, Lambda2",
                         "kappa_min": _round(float(k9.min())), "kappa_max": _round(float(k9.max())),
                         f"sigma_max_rel_kappa_le_{KAPPA_WELL:.0e}": _round(float(e9[well].max())) if well.any() else None,
                         f"events_kappa_le_{KAPPA_WELL:.0e}": int(well.sum()),
                         "sigma_max_rel_all": _round(float(e9.max()))}
    return out


def passes(name, e) -> bool:
    """The accuracy bar of a form on the sampled events.  FP64 forms: SNR
    1e-12, Fisher 1e-9 (normalised), no NaN sigma where the oracle has one,
    every sigma within the first-order bound of its event, and the
    well-conditioned block's sigmas within 1e-9.  Mixed form: SNR 5e-7,
    Fisher 1e-6 and sigma 1e-3 on every event with kappa < 1e12 (where the
    FP64 forms' own error stays far below 1e-3), a NaN counting as a miss."""
    if name == "batched_mixed":
        m = e[f"sigma_max_rel_kappa_lt_{KAPPA_MIXED:.0e}"]
        return (e["snr_max_rel"] <= 5e-7 and e["fisher_max_norm"] <= 1e-6 and m is not None and m <= 1e-3
                and e[f"sigma_nan_kappa_lt_{KAPPA_MIXED:.0e}"] == 0)
    b9 = e.get("block9", {})
    w = b9.get(f"sigma_max_rel_kappa_le_{KAPPA_WELL:.0e}")
    return (e["snr_max_rel"] <= 1e-12 and e["fisher_max_norm"] <= 1e-9 and e["sigma_nan_events"] == 0
            and e["sigma_within_first_order_bound"] == 1.0 and (w is None or w <= 1e-9))


def gradient_form(binding, synth, torch, args, timed) -> dict:
    """Forward (Fisher + inversion with ln det) and backward (adjoint) of
    J = sum ln SNR + sum ln det Gamma over the 10^4-event mixed BBH/BNS
    workload on five L sites, gradient along the 20 site parameters; each
    event's Fisher matrix has its kind's parameters (11 for BBH, 13 for BNS).
    Timed through a plan (the batched forward and backward over work items)
    and, for the backward alone, also with the one-workgroup-per-event
    adjoint."""
    from paper_2207_06910_amd import autodiff
    wl = synth.mixed1e4()
    dw = binding.DeviceWorkload(wl)
    xi = autodiff.site_parameters(dw)
    plan = binding.Plan(dw)                      # FP64, autotuned

    def step():
        x = xi.clone().requires_grad_(True)
        J = autodiff.network_fom(x, dw, plan=plan)
        J.backward()
        return x.grad

    for i in range(2):
        step()
    ms = timed(step, max(3, args.steps // 4))
    plan.set_sites(dw.sites)
    r = plan.run()
    inv = binding.invert(r["fisher"], r["status"], par_mask=dw.par_mask)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def kernel_ms(fn):
        fn()
        t = []
        for i in range(max(3, args.steps // 4)):
            ev[0].record(stream)
            fn()
            ev[1].record(stream)
            ev[1].synchronize()
            t.append(ev[0].elapsed_time(ev[1]))
        return float(np.mean(t))
    fwd = kernel_ms(lambda: plan.run())
    bwd = kernel_ms(lambda: plan.adjoint(inv["cov"], status=inv["status"]))
    bwd_plain = kernel_ms(lambda: binding.fisher_adjoint(dw, inv["cov"], status=inv["status"]))
    info = plan.info()
    plan.close()
    log(f"gradient (mixed1e4): {ms:.3f} ms per forward+backward through a plan; plan Fisher {fwd:.3f} ms, "
        f"plan adjoint {bwd:.3f} ms ({bwd / fwd:.2f}x the forward), one-workgroup-per-event adjoint "
        f"{bwd_plain:.3f} ms")
    fla = kernel_flops(wl, "adjoint")
    adj_tf = fla["total"] / (bwd * 1e-3) / 1e12
    return {"gradient_mixed1e4": {"workload": "mixed1e4: 10^4 events (60% BBH, 40% BNS), five L "
                                              "sites, 11 (BBH) / 13 (BNS) parameters, d/d(lat, lon, gamma, ln S0)",
                                  "grid_points": int(wl.npts.sum()),
                                  "ms_per_forward_backward": round(ms, 4),
                                  "plan_fisher_ms": round(fwd, 4),
                                  "adjoint_ms": round(bwd, 4),
                                  "adjoint_over_forward": round(bwd / fwd, 3),
                                  "adjoint_per_event_ms": round(bwd_plain, 4),
                                  "adjoint_roofline": {
                                      "bound": "alu", "achieved": round(adj_tf, 3), "peak": PEAK_FP64_TFLOPS,
                                      "unit": "TFLOP/s", "frac": round(adj_tf / PEAK_FP64_TFLOPS, 4),
                                      "flops_per_launch": fla["total"], "flops_per_point": fla["per_point"],
                                      "timed": "the whole backward call: set-up, work items, combine, reduce"},
                                  "chunk": info["chunk"],
                                  "events_per_s": round(wl.n / (ms * 1e-3), 1)}}


def catalogue_form(binding, synth, torch, args, timed, info) -> dict:
    """The batched FP64 form (same item length as on the BNS catalogue) on the 10^6-event BBH/BNS/NSBH catalogue, each
    event's Fisher matrix with its kind's parameters (11, 13 or 12)."""
    wl = synth.catalog1e6()
    dw = binding.DeviceWorkload(wl)
    plan = binding.Plan(dw, chunk=info["chunk"])
    out = {}
    plan.run(invert=True, out=out)
    ms = timed(lambda: plan.run(invert=True, out=out), 3)
    st = out["status"].cpu().numpy()
    pinfo = plan.info()
    plan.close()
    log(f"catalogue (catalog1e6): {ms:.3f} ms per step, {pinfo['n_items']} items, "
        f"inverted {int(np.sum(st == 0))}/{wl.n}")
    return {"batched_fp64_catalog1e6": {
        "workload": "catalog1e6: 10^6 events (60% BBH, 35% BNS, 5% NSBH), the BNS catalogue's "
                    "network (triangle + 2 L), 11 / 13 / 12 parameters by kind, 500-20000 points "
                    "from 2 Hz",
        "grid_points": int(wl.npts.sum()), "ms_per_step": round(ms, 3),
        "events_per_s": round(wl.n / (ms * 1e-3), 1), "n_items": pinfo["n_items"],
        "inverted": int(np.sum(st == 0)), "ill_conditioned_or_not_pd": int(np.sum((st & 6) != 0))}}


def bbh100_form(binding, synth, torch, args, timed) -> dict:
    """The small configuration: 100 BBH events, one L interferometer at the
    H1 site, no Earth rotation, 1000-point grids, 11 parameters; the same
    step (SNR and Fisher, then the inversion with the SVD fallback)."""
    wl = synth.bbh100()
    dw = binding.DeviceWorkload(wl)
    o1, o2 = {}, {}

    def step():
        r = binding.fisher(dw, out=o1)
        binding.covariance(r["fisher"], r["status"], method="cho_svd", out=o2)

    for i in range(3):
        step()
    ms = timed(step, max(5, args.steps))
    st = o2["status"].cpu().numpy()
    log(f"bbh100: {ms:.4f} ms per step, inverted {int(np.sum((st & ~32) == 0))}/{wl.n}")
    return {"plain_fp64_bbh100": {"workload": "bbh100: 100 BBH, one L interferometer (H1 site), no "
                                              "rotation, 1000 points from 10 Hz, 11 parameters",
                                  "ms_per_step": round(ms, 4), "events_per_s": round(wl.n / (ms * 1e-3), 1),
                                  "inverted": int(np.sum((st & ~32) == 0))}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chunk", type=int, default=0, help="batched form: fixed item length (0: autotune)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the detector-gradient and 10^6-event catalogue measurements")
    ap.add_argument("--skip", default="", metavar="LIST",
                    help="comma-separated measurements to leave out: covariance, strain, bbh100, "
                         "gradient, catalogue")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB device-to-device (a plain copy kernel of "
                         "known size, for calibrating HBM byte counters)")
    args = ap.parse_args()
    skip = {x.strip() for x in args.skip.split(",") if x.strip()}
    if args.no_extra:
        skip |= {"gradient", "catalogue"}
    unknown = skip - {"covariance", "strain", "bbh100", "gradient", "catalogue"}
    if unknown:
        ap.error(f"unknown --skip entries: {sorted(unknown)}")
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the path shards "
              f"events across GPUs with no exchange, so per-GPU throughput is the figure.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2207_06910_amd import binding, synth

    binding.load()
    torch.cuda.set_device(0)
    wl = synth.bns1e4()
    log(f"workload: {wl.n} events, {int(wl.npts.sum())} grid points, {wl.n_ifo} interferometers")
    dw = binding.DeviceWorkload(wl)
    P = wl.npar
    outf = {"fisher": torch.empty((P, P, wl.n), dtype=torch.float64, device="cuda"),
            "snr": torch.empty(wl.n, dtype=torch.float64, device="cuda"),
            "status": torch.empty(wl.n, dtype=torch.int32, device="cuda")}
    outi = {}

    # the paper's default inversion (sec. 4.1): Cholesky, an SVD where it fails
    def invert(F, status, out):
        return binding.covariance(F, status, method="cho_svd", out=out)

    def step():
        binding.fisher(dw, out=outf)
        invert(outf["fisher"], outf["status"], outi)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    # ---- plain form: one workgroup per event, ordinary launches
    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    plain_ms = timed(step, args.steps)
    log(f"plain: {args.steps} steps, {plain_ms:.3f} ms/step")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tf, ti = [], []
    for i in range(args.steps):
        ev[0].record(stream)
        binding.fisher(dw, out=outf)
        ev[1].record(stream)
        invert(outf["fisher"], outf["status"], outi)
        ev[2].record(stream)
        ev[2].synchronize()
        tf.append(ev[0].elapsed_time(ev[1]))
        ti.append(ev[1].elapsed_time(ev[2]))
    fisher_ms = float(np.mean(tf))
    invert_ms = float(np.mean(ti))
    st = outf["status"].cpu().numpy()
    sti = outi["status"].cpu().numpy()
    log(f"plain fisher kernel {fisher_ms:.3f} ms, invert kernel {invert_ms:.3f} ms, "
        f"Fisher status ok {int(np.sum(st == 0))}/{wl.n}, inverted {int(np.sum((sti & ~32) == 0))}/{wl.n} "
        f"({int(np.sum(sti == 32))} by SVD after a failed Cholesky)")

    def block9(F, status):
        r9 = binding.covariance(F, status, fixed=BLOCK_FIXED, method="cho")
        return r9["sigma"].cpu().numpy()

    plain_res = {"snr": outf["snr"].cpu().numpy(), "fisher": outf["fisher"].cpu().numpy(),
                 "sigma": outi["sigma"].cpu().numpy(), "sigma9": block9(outf["fisher"], outf["status"])}

    # ---- batched forms: work items (one workgroup each), one HIP graph per step
    def batched(mixed, chunk):
        plan = binding.Plan(dw, chunk=chunk, mixed=mixed, inv_method="cho_svd")   # 0: autotuned
        info = plan.info()
        outb = {}
        for i in range(args.warmup):
            plan.run(invert=True, out=outb)
        ms = timed(lambda: plan.run(invert=True, out=outb), args.steps)
        prof = binding.Plan(dw, chunk=info["chunk"], use_graph=False,
                            profile=True, mixed=mixed, inv_method="cho_svd")
        items = []
        outp = {}
        for i in range(args.steps):
            prof.run(invert=True, out=outp)
            items.append(prof.info()["items_ms"])
        prof.close()
        res = {k: outb[k].cpu().numpy() for k in ("snr", "fisher", "sigma", "status")}
        res["sigma9"] = block9(outb["fisher"], torch.zeros_like(outb["status"]))
        plan.close()
        sb = res["status"]
        tag = "mixed" if mixed else "FP64"
        log(f"batched {tag}: chunk {info['chunk']}, {info['n_items']} "
            f"items, {ms:.3f} ms/step, items kernel {float(np.mean(items)):.3f} ms, inverted "
            f"{int(np.sum((sb & ~32) == 0))}/{wl.n} ({int(np.sum(sb == 32))} by SVD after a failed Cholesky)")
        return ms, float(np.mean(items)), info, res

    batched_ms, items_ms, info, batched_res = batched(False, args.chunk)
    mixed_ms, mitems_ms, minfo, mixed_res = batched(True, args.chunk)

    cov_form = {}
    if "covariance" not in skip:
        # ---- covariance epilogue (gwf_covariance) on the plain form's Fisher matrices: the
        # paper's worked example (spins fixed, Gaussian priors of variance 2 pi^2 on the
        # angles, 90% sky area in square degrees) with the tidal deformabilities
        # marginalised over, inverted by the paper's default method (Cholesky, an SVD
        # where it fails)
        outc = {}
        ckw = dict(theta=dw.par[3].contiguous(), fixed=(9, 10), marg=(11, 12), sky_level=90.0,
                   units="SqDeg", prior={i: 1.0 / (2.0 * np.pi ** 2) for i in (3, 4, 5, 6, 8)},
                   method="cho_svd", out=outc)
        for i in range(2):
            binding.covariance(outf["fisher"], outf["status"], **ckw)
        tc = []
        for i in range(args.steps):
            ev[0].record(stream)
            binding.covariance(outf["fisher"], outf["status"], **ckw)
            ev[1].record(stream)
            ev[1].synchronize()
            tc.append(ev[0].elapsed_time(ev[1]))
        cov_ms = float(np.mean(tc))
        stc, skyc = outc["status"].cpu().numpy(), outc["sky"].cpu().numpy()
        log(f"covariance epilogue kernel {cov_ms:.3f} ms, inverted {int(np.sum(stc == 0))}/{wl.n} "
            f"(+{int(np.sum(stc == 32))} by SVD), median 90% sky area {float(np.median(skyc[stc == 0])):.3g} deg^2")
        def time_cov(**kw):
            o = {}
            for i in range(2):
                binding.covariance(outf["fisher"], outf["status"], out=o, **kw)
            t = []
            for i in range(args.steps):
                ev[0].record(stream)
                binding.covariance(outf["fisher"], outf["status"], out=o, **kw)
                ev[1].record(stream)
                ev[1].synchronize()
                t.append(ev[0].elapsed_time(ev[1]))
            return float(np.mean(t))
        # every matrix by SVD, with its eigen-decomposition (the paper's 'svd' and
        # CheckFisher), and every 13 x 13 matrix by the double-double Cholesky
        svd_ms = time_cov(method="svd", eigen=True)
        dd_ms = time_cov(method="cho_dd")
        log(f"SVD inversion with eigen-decomposition {svd_ms:.3f} ms, double-double Cholesky {dd_ms:.3f} ms")
        cov_form = {"covariance_epilogue": {
            "workload": "bns1e4 Fisher matrices: chi1z, chi2z fixed; Gaussian priors of variance 2 pi^2 "
                        "on theta, phi, iota, psi, Phicoal; Lambda1, Lambda2 marginalised; 90% sky area",
            "kernel": "invert_kernel<11>", "kernel_ms": round(cov_ms, 4),
            "events_per_s": round(wl.n / (cov_ms * 1e-3), 1), "inverted": int(np.sum(stc == 0)),
            "inverted_by_svd": int(np.sum(stc == 32)),
            "median_sky_deg2": round(float(np.median(skyc[stc == 0])), 4),
            "svd_with_eigen_ms": round(svd_ms, 4), "cho_dd_ms": round(dd_ms, 4)}}

    wave = {}
    if "strain" not in skip:
        # ---- strain output (gwf_waveform): HBM-bound, 16 B per point and interferometer
        ends = torch.cumsum(dw.npts.to(torch.int64), 0)
        offsets = ends - dw.npts.to(torch.int64)
        total = int(ends[-1].item())
        outw = {"h": torch.empty((wl.n_ifo, total), dtype=torch.complex128, device="cuda")}
        for mixed in (False, True):
            for i in range(2):
                binding.waveform(dw, offsets=offsets, total=total, out=outw, mixed=mixed)
            tw = []
            for i in range(max(3, args.steps // 4)):
                ev[0].record(stream)
                binding.waveform(dw, offsets=offsets, total=total, out=outw, mixed=mixed)
                ev[1].record(stream)
                ev[1].synchronize()
                tw.append(ev[0].elapsed_time(ev[1]))
            wave_ms = float(np.mean(tw))
            wave_bytes = 16.0 * wl.n_ifo * total + 8.0 * (13 * wl.n + 3 * wl.n)
            wave_gbs = wave_bytes / (wave_ms * 1e-3) / 1e9
            name = "waveform_mixed" if mixed else "waveform_fp64"
            log(f"{name} kernel {wave_ms:.3f} ms, {wave_bytes / 1e9:.2f} GB written, {wave_gbs:.0f} GB/s")
            wave[name] = {"kernel": "waveform_kernel<rot,tidal%s>" % (",mixed" if mixed else ""),
                          "kernel_ms": round(wave_ms, 4), "bytes": wave_bytes,
                          "achieved_GBs": round(wave_gbs, 1), "peak_GBs": PEAK_HBM_GBS,
                          "frac": round(wave_gbs / PEAK_HBM_GBS, 4),
                          "traffic": MEASURED_TRAFFIC.get("waveform_kernel<rot,tidal%s>" % (",mixed" if mixed else ""))}
        # the write ceiling of the same buffer: torch's own fills (a memset of
        # zeros and an elementwise fill kernel), timed the same way
        for name, fn in (("fill_zero", lambda: outw["h"].zero_()), ("fill_value", lambda: outw["h"].fill_(1.0))):
            fn()
            tw = []
            for i in range(max(3, args.steps // 4)):
                ev[0].record(stream)
                fn()
                ev[1].record(stream)
                ev[1].synchronize()
                tw.append(ev[0].elapsed_time(ev[1]))
            fms = float(np.mean(tw))
            fbytes = 16.0 * wl.n_ifo * total
            log(f"{name} of the strain buffer {fms:.3f} ms, {fbytes / (fms * 1e-3) / 1e9:.0f} GB/s")
            wave["waveform_fp64"][name + "_ms"] = round(fms, 4)
            wave["waveform_fp64"][name + "_GBs"] = round(fbytes / (fms * 1e-3) / 1e9, 1)
        del outw
        # ---- strain derivatives (gwf_waveform_deriv) on the first 10^3 events:
        # 16 B per point, interferometer and parameter (13), about 10 GB
        nd = min(1000, wl.n)
        wd = wl.subset(np.arange(nd))
        dwd = binding.DeviceWorkload(wd)
        endd = torch.cumsum(dwd.npts.to(torch.int64), 0)
        offd, totd = endd - dwd.npts.to(torch.int64), int(endd[-1].item())
        outd = {"dh": torch.empty((13, wd.n_ifo, totd), dtype=torch.complex128, device="cuda")}
        for i in range(2):
            binding.waveform_deriv(dwd, offsets=offd, total=totd, out=outd)
        td = []
        for i in range(max(3, args.steps // 4)):
            ev[0].record(stream)
            binding.waveform_deriv(dwd, offsets=offd, total=totd, out=outd)
            ev[1].record(stream)
            ev[1].synchronize()
            td.append(ev[0].elapsed_time(ev[1]))
        der_ms = float(np.mean(td))
        der_bytes = 16.0 * 13 * wd.n_ifo * totd + 8.0 * (13 * nd + 3 * nd)
        der_gbs = der_bytes / (der_ms * 1e-3) / 1e9
        log(f"waveform_deriv kernel {der_ms:.3f} ms, {der_bytes / 1e9:.2f} GB written, {der_gbs:.0f} GB/s")
        wave["waveform_deriv_fp64"] = {"kernel": "waveform_deriv_kernel<rot,tidal>",
                                       "workload": f"first {nd} events of bns1e4, 13 parameters",
                                       "kernel_ms": round(der_ms, 4), "bytes": der_bytes,
                                       "achieved_GBs": round(der_gbs, 1), "peak_GBs": PEAK_HBM_GBS,
                                       "frac": round(der_gbs / PEAK_HBM_GBS, 4),
                                       "traffic": MEASURED_TRAFFIC.get("waveform_deriv_kernel<rot,tidal>")}
        del outd

    extra = {} if "bbh100" in skip else bbh100_form(binding, synth, torch, args, timed)
    if "gradient" not in skip:
        extra.update(gradient_form(binding, synth, torch, args, timed))
    if "catalogue" not in skip:
        extra.update(catalogue_form(binding, synth, torch, args, timed, info))

    cpu, errs = None, {}
    if not args.no_cpu_baseline:
        log(f"cpu baseline on {args.cpu_sample} events ...")
        cpu, ref = cpu_baseline(wl, args.cpu_sample)
        log(f"cpu baseline {cpu['value']:.3f} events/s")
        errs = {"plain_fp64": error_report(plain_res, ref),
                "batched_fp64": error_report(batched_res, ref),
                "batched_mixed": error_report(mixed_res, ref)}
        for k, v in errs.items():
            log(f"{k} vs oracle: {v}")

    if args.copy_calibration > 0:
        nd = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nd, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for i in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.copy_calibration} MiB")

    # the reported form: the fastest one that meets its accuracy bar on the
    # sampled events (passes()); without the oracle sample only the FP64
    # forms are eligible
    def eligible(name):
        return passes(name, errs[name]) if name in errs else name != "batched_mixed"

    cands = [("plain_fp64", plain_ms, "fisher_kernel<tidal,rot>", fisher_ms),
             ("batched_fp64", batched_ms, "items_kernel<tidal,rot>", items_ms),
             ("batched_mixed", mixed_ms, "items_kernel<tidal,rot,mixed>", mitems_ms)]
    ok = [c for c in cands if eligible(c[0])]
    if not ok:
        log("no form met its accuracy bar; reporting the plain FP64 form")
        ok = cands[:1]
    form, ms, kname, kms = min(ok, key=lambda c: c[1])

    def roofline_of(kname, kms):
        fl = kernel_flops(wl, "items_mixed" if "mixed" in kname else "items")
        achieved = fl["total"] / (kms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": MEASURED_TRAFFIC.get(kname), "traffic_unit": "bytes per launch",
                "kernel": kname, "kernel_ms": round(kms, 4), "flops_per_launch": fl["total"],
                "flops_per_point": fl["per_point"], "flops_mfma_per_launch": fl["mfma"],
                "flops_model": "executed FP64 flops of the kernel's instruction stream (FMA = 2), "
                               "VALU and MFMA, confirmed by SQ_INSTS_VALU_FLOPS_FP64 and "
                               "SQ_INSTS_VALU_MFMA_MOPS_F64",
                "dense_count_frac": round(fl["dense"] / (kms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
                "valu_busy": valu_busy(kname, kms)}
    roofline = roofline_of(kname, kms)
    # the fastest form at the paper's precision, beside the headline
    f64 = min([c for c in ok if c[0] != "batched_mixed"] or cands[:2], key=lambda c: c[1])
    fp64_line = {"form": f64[0], "value": round(wl.n / (f64[1] * 1e-3), 1), "unit": "events/s",
                 "ms_per_step": round(f64[1], 4), "roofline": roofline_of(f64[2], f64[3])}

    value = wl.n / (ms * 1e-3)
    forms = {"plain_fp64": {"events_per_s": round(wl.n / (plain_ms * 1e-3), 1),
                            "ms_per_step": round(plain_ms, 4), "fisher_ms": round(fisher_ms, 4),
                            "invert_ms": round(invert_ms, 4)},
             "batched_fp64": {"events_per_s": round(wl.n / (batched_ms * 1e-3), 1),
                              "ms_per_step": round(batched_ms, 4), "items_ms": round(items_ms, 4),
                              "chunk": info["chunk"],
                              "n_items": info["n_items"], "graph": True},
             "batched_mixed": {"events_per_s": round(wl.n / (mixed_ms * 1e-3), 1),
                               "ms_per_step": round(mixed_ms, 4), "items_ms": round(mitems_ms, 4),
                               "chunk": minfo["chunk"],
                               "n_items": minfo["n_items"], "graph": True}}
    for k, v in errs.items():
        forms[k]["errors_vs_oracle"] = v
    forms.update(cov_form)
    forms.update(wave)
    forms.update(extra)
    out = {
        "metric": "Fisher events/s (BNS, 3-det, Earth-rot) plain FP64 vs mixed/batched @tol",
        "value": round(value, 1), "unit": "events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64/f32" if form == "batched_mixed" else "f64", "data": "synthetic",
        "config": {"workload": "bns1e4: 10^4 BNS (m1,m2 in 1.1-2.2 Msun, tides, aligned spins), "
                               "triangle + 2 L sites (5 interferometers), Earth rotation, 13 "
                               "parameters, log grids 2 Hz to f_cut of 2000-20000 points",
                   "events": wl.n, "grid_points": int(wl.npts.sum()), "form": form},
        "forms": forms,
        "roofline": roofline,
        "fp64": fp64_line,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""CPU: the oracle and the host build of the kernels' per-point mathematics
under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/sanitize_main.cpp links both, built with clang's
-fsanitize=address,undefined (no recovery: the first report ends the run
with a nonzero status), runs them on small seeded workloads (BNS events on
the five-interferometer network with rotation and tides; BBH events on one
L site), and writes their outputs.  The test asks for a clean exit and for
outputs equal, to rounding, to those of the ordinary builds, so the
instrumented run took the same paths."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2207_06910_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1", "-std=c++17"]


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(CXX):
        pytest.skip("clang++ of the ROCm toolchain not found")
    d = tmp_path_factory.mktemp("sanitize")
    host_san = ["-fsanitize=address,undefined"]
    steps = [
        [CXX, *host_san, *SAN, "-Wno-unknown-pragmas", "-c", os.path.join(ROOT, "oracle", "gwf_oracle.cpp"),
         "-o", str(d / "oracle.o")],
        # host side only: the kernels' mathematics compiled for the CPU, no device code
        [CXX, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "--rocm-path=/opt/rocm",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *SAN, "-w", "-c",
         os.path.join(HERE, "model_host", "model_host.hip"), "-o", str(d / "model_host.o")],
        [CXX, *host_san, *SAN, "-c", os.path.join(HERE, "sanitize", "sanitize_main.cpp"), "-o", str(d / "main.o")],
        [CXX, *host_san, *SAN, str(d / "oracle.o"), str(d / "model_host.o"), str(d / "main.o"),
         "-o", str(d / "sanitize_main")],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
    return d / "sanitize_main"


def _workloads():
    bns = synth.bns1e4(n=40).subset(np.array([3, 17, 31])).with_npts(300)
    bbh = synth.bbh100(n=4, npts=200)
    return [("bns", bns), ("bbh", bbh)]


def _run(exe, wl, gbar, tmp):
    P = gbar.shape[0]
    sites = wl.site_array()
    with open(tmp / "in.bin", "wb") as f:
        np.array([wl.n, len(sites), wl.flags, P], dtype=np.int64).tofile(f)
        np.ascontiguousarray(wl.par[:13], dtype=np.float64).tofile(f)
        np.ascontiguousarray(sites, dtype=np.float64).tofile(f)
        np.ascontiguousarray(wl.fmin, dtype=np.float64).tofile(f)
        np.ascontiguousarray(wl.npts, dtype=np.int32).tofile(f)
        np.ascontiguousarray(gbar, dtype=np.float64).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(tmp / "in.bin"), str(tmp / "out.bin")], capture_output=True, text=True,
                       env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized run ok" in r.stdout
    return np.fromfile(tmp / "out.bin", dtype=np.float64)


def _close(a, b, tol):
    scale = np.abs(b).max()
    assert np.all(np.isfinite(a))
    assert np.abs(a - b).max() <= tol * scale, (np.abs(a - b).max(), scale)


@pytest.mark.parametrize("name", ["bns", "bbh"])
def test_sanitized_oracle_and_host_math(exe, orc, tmp_path, name):
    import model_host

    wl = dict(_workloads())[name]
    n = wl.n
    ref = orc.fisher(wl)
    F = ref["fisher"]
    P = F.shape[0]
    d = np.sqrt(np.einsum("iie->ie", F))
    gbar = np.random.default_rng(6).normal(size=(P, P, n)) / (d[:, None, :] * d[None, :, :])
    out = _run(exe, wl, gbar, tmp_path)

    ni = orc.n_ifo(wl.site_array())
    total = int(wl.npts.sum())
    offsets = np.concatenate([[0], np.cumsum(wl.npts)[:-1]]).astype(np.int64)
    sizes = [n, P * P * n, ni * total * 2, P * ni * total * 2, 2 * n, 2 * P * P * n, n, P * P * n,
             n * len(wl.sites) * 4, n]
    assert out.size == sum(sizes)
    parts = np.split(out, np.cumsum(sizes)[:-1])
    snr, Fo, h, dh, t_s, t_F, m_snr, m_F, m_adj, cond = parts

    _close(snr, ref["snr"], 1e-13)
    _close(Fo.reshape(P, P, n), F, 1e-12)
    h_ref = orc.waveform(wl, offsets, total)
    _close(h.view(np.complex128).reshape(h_ref.shape), h_ref, 1e-10)
    dh_ref = orc.waveform_derivs(wl, offsets, total)
    _close(dh.view(np.complex128).reshape(dh_ref.shape), dh_ref, 1e-10)
    tan = orc.fisher_tangent(wl, 0, 1)
    _close(t_s.reshape(2, n), np.asarray(tan["snr2"]), 1e-12)
    _close(t_F.reshape(2, P, P, n), np.asarray(tan["fisher"]), 1e-12)

    mh = model_host.fisher(wl)
    _close(m_snr, mh["snr"], 1e-13)
    _close(m_F.reshape(P, P, n), mh["fisher"], 1e-12)
    adj = model_host.adjoint(wl, gbar, w_snr=0.7, w_fisher=1.3)
    _close(m_adj.reshape(adj.shape), adj, 1e-11)
    c_ref, _ = model_host.jacobi_cond(F)
    # same Jacobi sweeps; at kappa ~ 1e12 the two builds' rounding (FMA contraction
    # differs between -O1 and -O2) moves the smallest singular value by ~kappa u
    np.testing.assert_allclose(cond, c_ref, rtol=1e-6)

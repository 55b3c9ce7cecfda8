"""TEST ONLY: host build of the kernels' per-point mathematics (see model_host.hip)."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "model_host.hip")
LIB = os.path.join(HERE, "libmodel_host.so")
DEPS = [SRC, os.path.join(HERE, "..", "..", "paper_2207_06910_amd", "csrc", "gwf_model.hpp"),
        os.path.join(HERE, "..", "..", "paper_2207_06910_amd", "csrc", "gwf_adjoint.hpp"),
        os.path.join(HERE, "..", "..", "paper_2207_06910_amd", "csrc", "gwf_invert.hpp"),
        os.path.join(HERE, "..", "..", "paper_2207_06910_amd", "csrc", "gwf_dd.hpp"),
        os.path.join(HERE, "..", "..", "paper_2207_06910_amd", "csrc", "gwf_arith.hpp")]
_lib = None


def load():
    global _lib
    if _lib is None:
        stale = not os.path.exists(LIB) or any(os.path.getmtime(d) > os.path.getmtime(LIB) for d in DEPS)
        if stale:
            subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared",
                                   "--offload-arch=gfx950", SRC, "-o", LIB + ".tmp"],
                                  stderr=subprocess.DEVNULL)
            os.replace(LIB + ".tmp", LIB)
        _lib = ctypes.CDLL(LIB)
    return _lib


def fisher(wl, flags=None):
    lib = load()
    flags = wl.flags if flags is None else flags
    P = 13 if wl.flags & 2 else 11
    n = wl.n
    par = np.ascontiguousarray(wl.par, dtype=np.float64)
    sites = np.ascontiguousarray(wl.site_array())
    fmin = np.ascontiguousarray(wl.fmin, dtype=np.float64)
    fmax = None if wl.fmax is None else np.ascontiguousarray(wl.fmax, dtype=np.float64)
    npts = np.ascontiguousarray(wl.npts, dtype=np.int32)
    F = np.zeros((P, P, n))
    snr = np.zeros(n)
    st = np.zeros(n, dtype=np.int32)
    P_ = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    lib.model_fisher_host(ctypes.c_int64(n), P_(par), ctypes.c_int64(n), P_(fmin), P_(fmax), P_(npts),
                          ctypes.c_int(len(sites)), P_(sites), ctypes.c_uint32(flags), P_(F),
                          P_(snr), P_(st))
    return {"fisher": F, "snr": snr, "status": st}


def adjoint(wl, gbar, w_snr=1.0, w_fisher=1.0):
    """Per-event gradient terms grad_event[N][n_site][4] of the host build."""
    lib = load()
    n = wl.n
    par = np.ascontiguousarray(wl.par, dtype=np.float64)
    sites = np.ascontiguousarray(wl.site_array())
    fmin = np.ascontiguousarray(wl.fmin, dtype=np.float64)
    fmax = None if wl.fmax is None else np.ascontiguousarray(wl.fmax, dtype=np.float64)
    npts = np.ascontiguousarray(wl.npts, dtype=np.int32)
    G = np.ascontiguousarray(gbar, dtype=np.float64)
    out = np.zeros((n, len(sites), 4))
    P_ = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    lib.model_adjoint_host(ctypes.c_int64(n), P_(par), ctypes.c_int64(n), P_(fmin), P_(fmax), P_(npts),
                           ctypes.c_int(len(sites)), P_(sites), ctypes.c_uint32(wl.flags), P_(G),
                           ctypes.c_double(w_snr), ctypes.c_double(w_fisher), P_(out))
    return out


def jacobi_partner(M, j, t):
    return int(load().model_jacobi_partner(ctypes.c_int(M), ctypes.c_int(j), ctypes.c_int(t)))


def jacobi_cond(F):
    """Condition numbers of F [P][P][N] by the inversion kernel's one-sided
    Jacobi (P in 2, 5, 9, 11, 13), and the sweeps it took."""
    lib = load()
    P, _, n = F.shape
    F = np.ascontiguousarray(F, dtype=np.float64)
    cond = np.zeros(n)
    sweeps = np.zeros(n, dtype=np.int32)
    P_ = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.model_jacobi_cond_host(ctypes.c_int(P), ctypes.c_int64(n), P_(F), P_(cond), P_(sweeps))
    assert rc == 0, "unsupported size"
    return cond, sweeps


def dd_op(op, a, b=(0.0, 0.0)):
    """The inversion's double-double primitive `op` (0 add, 1 sub, 2 mul,
    3 mul swapped, 4 div, 5 sqrt) on (hi, lo) pairs; returns (hi, lo)."""
    lib = load()
    x = np.array(a, dtype=np.float64)
    y = np.array(b, dtype=np.float64)
    o = np.zeros(2)
    P_ = lambda v: v.ctypes.data_as(ctypes.c_void_p)
    lib.model_dd(ctypes.c_int(op), P_(x), P_(y), P_(o))
    return float(o[0]), float(o[1])

"""TEST INFRASTRUCTURE ONLY -- ctypes front end of the C++ oracle.

Builds ``liboracle.so`` from ``gwf_oracle.cpp`` with g++ (no fast-math, so
IEEE semantics are kept) and exposes its entry points on numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gwf_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

FLAG_EARTH_ROT = 1
FLAG_TIDAL = 2
FLAG_ECC = 8

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_L = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle (always when force; otherwise only if missing)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        lib.orc_cut_frequency.restype = ctypes.c_double
        lib.orc_psd.restype = ctypes.c_double
        lib.orc_delay.restype = ctypes.c_double
        lib.orc_fisher.argtypes = [ctypes.c_int64, _D, ctypes.c_int64, _D, ctypes.c_int, _D, _D, _D,
                                   _I, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]
        lib.orc_waveform.argtypes = [ctypes.c_int64, _D, ctypes.c_int64, _D, ctypes.c_int, _D, _D, _D,
                                     _I, ctypes.c_int, ctypes.c_int, _L, ctypes.c_int64, _D]
        lib.orc_waveform_deriv.argtypes = lib.orc_waveform.argtypes
        lib.orc_set_explicit_grid.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_set_psd_tables.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_noise_weight.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         _D, _D, _D]
        lib.orc_fisher_tangent.argtypes = [ctypes.c_int64, _D, ctypes.c_int64, _D, ctypes.c_int, _D,
                                           _D, _D, _I, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, _D, _D]
        lib.orc_strain.argtypes = [_D, ctypes.c_double, ctypes.c_int, _D, ctypes.c_int, _D,
                                   ctypes.c_int, _D, _D]
        lib.orc_strain_cstep.argtypes = [_D, ctypes.c_double, ctypes.c_int, _D, ctypes.c_int, _D,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_double, _D]
        lib.orc_strain_plain.argtypes = [_D, ctypes.c_double, ctypes.c_double, ctypes.c_int, _D,
                                         ctypes.c_int, _D, ctypes.c_int, _D]
        lib.orc_phase_tau.argtypes = [_D, ctypes.c_int, ctypes.c_int, _D, _D, _D]
        lib.orc_phase_cstep_f.argtypes = [_D, ctypes.c_int, ctypes.c_int, _D, ctypes.c_double, _D]
        lib.orc_phase_cstep_par.argtypes = [_D, ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, ctypes.c_double, _D]
        lib.orc_set_eccentricity.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.orc_antenna.argtypes = [ctypes.c_double] * 7 + [_D, _D]
        lib.orc_delay.argtypes = [ctypes.c_double] * 4
        lib.orc_cut_frequency.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_psd.argtypes = [ctypes.c_double] * 3
        lib.orc_grid.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _D, _D]
        lib.orc_constants.argtypes = [_D]
        lib.orc_n_ifo.argtypes = [ctypes.c_int, _D]
        lib.orc_ifos.argtypes = [ctypes.c_int, _D, _D]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_D)


def n_params(flags):
    """Fisher parameters: 11, the two deformabilities with FLAG_TIDAL, and
    e0 (last) with FLAG_ECC."""
    return 11 + (2 if flags & FLAG_TIDAL else 0) + (1 if flags & FLAG_ECC else 0)


def _par15(par):
    """One event's parameters as the oracle takes them: the 13 rows, e0 and
    the reference frequency of e0 (0: the first frequency of the list or
    grid); a 13-vector is padded with zeros."""
    p = np.zeros(15)
    a = np.asarray(par, dtype=np.float64).ravel()
    p[:len(a)] = a
    return p


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def constants() -> dict:
    out = np.zeros(6)
    load().orc_constants(_p(out))
    return dict(zip(["T_SUN", "GPC_S", "OMEGA_E", "R_EARTH_S", "EULER_GAMMA", "PI"], out))


def cut_frequency(Mc, eta):
    return load().orc_cut_frequency(float(Mc), float(eta))


def psd(S0, f0, f):
    return load().orc_psd(float(S0), float(f0), float(f))


def grid(fmin, fmax, n):
    f = np.zeros(n)
    w = np.zeros(n)
    load().orc_grid(float(fmin), float(fmax), int(n), _p(f), _p(w))
    return f, w


def n_ifo(sites):
    s = _f64(sites)
    return load().orc_n_ifo(len(s), _p(s))


def ifos(sites):
    s = _f64(sites)
    out = np.zeros((n_ifo(s), 4))
    load().orc_ifos(len(s), _p(s), _p(out))
    return out


def antenna(lat, gamma, zeta, lst, theta, phi, psi):
    fp = ctypes.c_double()
    fx = ctypes.c_double()
    load().orc_antenna(lat, gamma, zeta, lst, theta, phi, psi, ctypes.byref(fp), ctypes.byref(fx))
    return fp.value, fx.value


def delay(lat, lst, theta, phi):
    return load().orc_delay(lat, lst, theta, phi)


def phase_tau(par13, f, flags=0):
    par = _par15(par13)
    f = _f64(f)
    psi = np.zeros_like(f)
    tau = np.zeros_like(f)
    load().orc_phase_tau(_p(par), flags, len(f), _p(f), _p(psi), _p(tau))
    return psi, tau


def phase_dpsi_df_cstep(par13, f, flags=0, h=1e-30):
    par = _par15(par13)
    f = _f64(f)
    out = np.zeros_like(f)
    load().orc_phase_cstep_f(_p(par), flags, len(f), _p(f), h, _p(out))
    return out


def phase_cstep_par(par, f, flags, j, h=1e-30):
    """d Psi_PN / d (slot j) at fixed frequencies by complex step (the
    eccentric term included under FLAG_ECC)."""
    par = _par15(par)
    f = _f64(f)
    out = np.zeros_like(f)
    load().orc_phase_cstep_par(_p(par), flags, int(j), len(f), _p(f), h, _p(out))
    return out


def strain(par13, sites, f, flags, tc_s=0.0, derivs=True):
    """h[n_ifo][nf] complex and, if derivs, dh[n_ifo][nf][P] complex."""
    par = _par15(par13)
    s = _f64(sites)
    f = _f64(f)
    ni = n_ifo(s)
    P = n_params(flags)
    h = np.zeros((ni, len(f), 2))
    dh = np.zeros((ni, len(f), P, 2)) if derivs else None
    load().orc_strain(_p(par), float(tc_s), len(s), _p(s), len(f), _p(f), flags, _p(h), _p(dh))
    hc = h[..., 0] + 1j * h[..., 1]
    if not derivs:
        return hc
    return hc, dh[..., 0] + 1j * dh[..., 1]


def strain_cstep(par13, sites, f, flags, j, step=1e-30, tc_s=0.0):
    par = _par15(par13)
    s = _f64(sites)
    f = _f64(f)
    out = np.zeros((n_ifo(s), len(f), 2))
    load().orc_strain_cstep(_p(par), float(tc_s), len(s), _p(s), len(f), _p(f), flags, int(j),
                            float(step), _p(out))
    return out[..., 0] + 1j * out[..., 1]


def strain_plain(par13, sites, f, flags, tc_s=0.0, dt=0.0):
    par = _par15(par13)
    s = _f64(sites)
    f = _f64(f)
    out = np.zeros((n_ifo(s), len(f), 2))
    load().orc_strain_plain(_p(par), float(tc_s), float(dt), len(s), _p(s), len(f), _p(f), flags,
                            _p(out))
    return out[..., 0] + 1j * out[..., 1]


class _grid:
    """While active, the workload-level drivers use wl.grid_f (explicit
    frequencies, trapezoid weights from their differences) in place of the
    log descriptors."""

    def __init__(self, wl):
        g = getattr(wl, "grid_f", None)
        self.f = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        self.off = None if g is None else np.ascontiguousarray(wl.grid_offsets(), dtype=np.int64)

    def __enter__(self):
        if self.f is not None:
            load().orc_set_explicit_grid(self.off.ctypes.data_as(ctypes.c_void_p),
                                         self.f.ctypes.data_as(ctypes.c_void_p))
        return self

    def __exit__(self, *exc):
        if self.f is not None:
            load().orc_set_explicit_grid(None, None)
        return False


class _ecc:
    """While active, the workload's eccentricities (wl.ecc) and their
    reference frequencies (wl.f_ref_ecc, or None: each grid's first
    frequency) are the events' e0 and f_ref."""

    def __init__(self, wl):
        e = getattr(wl, "ecc", None)
        fr = getattr(wl, "f_ref_ecc", None)
        self.e = None if e is None else np.ascontiguousarray(e, dtype=np.float64)
        self.fr = None if fr is None else np.ascontiguousarray(fr, dtype=np.float64)

    def __enter__(self):
        if self.e is not None:
            load().orc_set_eccentricity(self.e.ctypes.data,
                                        None if self.fr is None else self.fr.ctypes.data)
        return self

    def __exit__(self, *exc):
        if self.e is not None:
            load().orc_set_eccentricity(None, None)
        return False


class _tables:
    """While active, the sites' sampled noise curves (psd_kind 1 = PSD, 2 =
    ASD, with psd_f and psd_S) are used in place of the analytic PSD."""

    def __init__(self, sites):
        self.sites = list(sites)
        self.kind = np.array([int(getattr(s, "psd_kind", 0)) for s in self.sites], dtype=np.int32)
        self.f = [None if k == 0 else np.ascontiguousarray(s.psd_f, dtype=np.float64)
                  for k, s in zip(self.kind, self.sites)]
        self.S = [None if k == 0 else np.ascontiguousarray(s.psd_S, dtype=np.float64)
                  for k, s in zip(self.kind, self.sites)]

    def __enter__(self):
        if self.kind.any():
            ns = len(self.sites)
            self.n = np.array([0 if f is None else len(f) for f in self.f], dtype=np.int64)
            self.fp = (ctypes.c_void_p * ns)(*[None if f is None else f.ctypes.data for f in self.f])
            self.Sp = (ctypes.c_void_p * ns)(*[None if x is None else x.ctypes.data for x in self.S])
            load().orc_set_psd_tables(ns, self.kind.ctypes.data, self.n.ctypes.data,
                                      ctypes.cast(self.fp, ctypes.c_void_p), ctypes.cast(self.Sp, ctypes.c_void_p))
        return self

    def __exit__(self, *exc):
        if self.kind.any():
            load().orc_set_psd_tables(0, None, None, None, None)
        return False


def noise_weight(site, f, w):
    """4 w / S_n(f) of one site's noise curve (analytic or sampled) at
    frequencies f with trapezoid weights w; zero where a sampled curve does
    not reach."""
    f = _f64(f)
    w = _f64(w)
    out = np.zeros_like(f)
    with _tables([site]):
        load().orc_noise_weight(float(site.S0), float(site.f0), 0, len(f), _p(f), _p(w), _p(out))
    return out


def restrict_rows(F, par_mask):
    """Each event's Fisher matrix over its own parameter set: in F[P][P][N]
    (in place), the rows and columns of parameters outside event e's set
    (bit i of par_mask[e] clear) are set to 0."""
    P = F.shape[0]
    for i in range(P):
        out = ((np.asarray(par_mask, dtype=np.int64) >> i) & 1) == 0
        F[i, :, out] = 0.0
        F[:, i, out] = 0.0
    return F


def fisher(wl, want_fisher=True, per_ifo=False, nthreads=0):
    """SNR (and Fisher) of a synthetic workload, as a dict of numpy arrays:
    snr[N], snr_ifo[n_ifo][N], fisher[P][P][N], fisher_ifo[n_ifo][P][P][N].
    With wl.active (the duty factor's on/off draws, uint8 [n_ifo][N]) the
    interferometers that are off for an event are left out of its sums; with
    wl.par_mask (uint32 [N]) each event's matrix covers its own parameters
    only (restrict_rows)."""
    par = _f64(wl.par)
    n = par.shape[1]
    s = _f64(wl.site_array())
    ni = n_ifo(s)
    P = n_params(wl.flags)
    fmin = _f64(wl.fmin)
    fmax = None if wl.fmax is None else _f64(wl.fmax)
    npts = np.ascontiguousarray(wl.npts, dtype=np.int32)
    tc = None if wl.tc_s is None else _f64(wl.tc_s)
    snr = np.zeros(n)
    snr_ifo = np.zeros((ni, n))
    F = np.zeros((P, P, n)) if want_fisher else None
    Fi = np.zeros((ni, P, P, n)) if (want_fisher and per_ifo) else None
    act = getattr(wl, "active", None)
    act = None if act is None else np.ascontiguousarray(act, dtype=np.uint8)
    with _grid(wl), _tables(wl.sites), _ecc(wl):
        load().orc_fisher(n, _p(par), n, _p(tc), len(s), _p(s), _p(fmin), _p(fmax),
                          npts.ctypes.data_as(_I), None if act is None else act.ctypes.data_as(ctypes.c_void_p),
                          wl.flags, int(nthreads), _p(snr), _p(snr_ifo), _p(F), _p(Fi))
    pm = getattr(wl, "par_mask", None)
    if pm is not None and want_fisher:
        restrict_rows(F, pm)
        if Fi is not None:
            for d in range(ni):
                restrict_rows(Fi[d], pm)
    out = {"snr": snr, "snr_ifo": snr_ifo}
    if want_fisher:
        out["fisher"] = F
    if Fi is not None:
        out["fisher_ifo"] = Fi
    return out


def waveform(wl, offsets=None, total=None, nthreads=0):
    """Strain of every event of a workload at every interferometer on its own
    grid, as complex h[n_ifo][total]; event e fills columns offsets[e] ..
    offsets[e]+npts[e]-1 (default: packed in event order, total = sum npts)."""
    par = _f64(wl.par)
    n = par.shape[1]
    s = _f64(wl.site_array())
    ni = n_ifo(s)
    npts = np.ascontiguousarray(wl.npts, dtype=np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum(npts, dtype=np.int64)[:-1]])
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    if total is None:
        total = int(np.max(offsets + npts))
    fmin = _f64(wl.fmin)
    fmax = None if wl.fmax is None else _f64(wl.fmax)
    tc = None if wl.tc_s is None else _f64(wl.tc_s)
    h = np.zeros((ni, total, 2))
    with _grid(wl), _ecc(wl):
        load().orc_waveform(n, _p(par), n, _p(tc), len(s), _p(s), _p(fmin), _p(fmax),
                            npts.ctypes.data_as(_I), wl.flags, int(nthreads),
                            offsets.ctypes.data_as(_L), int(total), _p(h))
    return h[..., 0] + 1j * h[..., 1]


def waveform_derivs(wl, offsets=None, total=None, nthreads=0):
    """Derivatives of the strain with respect to the P parameters (the
    Fisher matrix's rows, in its units), as complex dh[P][n_ifo][total] laid
    out as waveform(); with wl.par_mask the rows outside an event's set are
    0 there."""
    par = _f64(wl.par)
    n = par.shape[1]
    s = _f64(wl.site_array())
    ni = n_ifo(s)
    P = n_params(wl.flags)
    npts = np.ascontiguousarray(wl.npts, dtype=np.int32)
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum(npts, dtype=np.int64)[:-1]])
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    if total is None:
        total = int(np.max(offsets + npts))
    fmin = _f64(wl.fmin)
    fmax = None if wl.fmax is None else _f64(wl.fmax)
    tc = None if wl.tc_s is None else _f64(wl.tc_s)
    dh = np.zeros((P, ni, total, 2))
    with _grid(wl), _ecc(wl):
        load().orc_waveform_deriv(n, _p(par), n, _p(tc), len(s), _p(s), _p(fmin), _p(fmax),
                                  npts.ctypes.data_as(_I), wl.flags, int(nthreads),
                                  offsets.ctypes.data_as(_L), int(total), _p(dh))
    out = dh[..., 0] + 1j * dh[..., 1]
    pm = getattr(wl, "par_mask", None)
    if pm is not None:
        for e in range(n):
            for r in range(P):
                if not (int(pm[e]) >> r) & 1:
                    out[r, :, offsets[e]:offsets[e] + npts[e]] = 0.0
    return out


def fisher_tangent(wl, site, which, nthreads=0):
    """SNR^2 and Fisher matrices of a workload with their derivatives along
    one detector parameter (which: 0 latitude, 1 longitude, 2 arm angle,
    3 ln S0, of site `site`): snr2[2][N], fisher[2][P][P][N], index 0 the
    value and 1 the derivative."""
    par = _f64(wl.par)
    n = par.shape[1]
    s = _f64(wl.site_array())
    P = n_params(wl.flags)
    fmin = _f64(wl.fmin)
    fmax = None if wl.fmax is None else _f64(wl.fmax)
    npts = np.ascontiguousarray(wl.npts, dtype=np.int32)
    tc = None if wl.tc_s is None else _f64(wl.tc_s)
    snr2 = np.zeros((2, n))
    F = np.zeros((2, P, P, n))
    act = getattr(wl, "active", None)
    act = None if act is None else np.ascontiguousarray(act, dtype=np.uint8)
    with _grid(wl), _tables(wl.sites), _ecc(wl):
        load().orc_fisher_tangent(n, _p(par), n, _p(tc), len(s), _p(s), _p(fmin), _p(fmax),
                                  npts.ctypes.data_as(_I), None if act is None else act.ctypes.data_as(ctypes.c_void_p),
                                  wl.flags, int(nthreads), int(site), int(which), _p(snr2), _p(F))
    pm = getattr(wl, "par_mask", None)
    if pm is not None:
        restrict_rows(F[0], pm)
        restrict_rows(F[1], pm)
    return {"snr2": snr2, "fisher": F}

"""Thin Python binding of libgwf (include/gwf.h): argument marshalling only.

Every computation runs in the HIP kernels of ``libgwf.so``; PyTorch only
provides device memory and the stream.  The library must have been built
(``python -m paper_2207_06910_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgwf.so")

GWF_OK, GWF_E_INVALID_ARG, GWF_E_UNSUPPORTED, GWF_E_HIP, GWF_E_NOMEM = 0, 1, 2, 3, 4
EV_INVALID_PARAM, EV_NOT_PD, EV_ILL_COND, EV_NONFINITE, EV_SKIPPED_SNR = 1, 2, 4, 8, 16
EARTH_ROT, TIDAL, MIXED, ECCENTRIC = 1, 2, 4, 8
SHAPE_L, SHAPE_T = 0, 1
PSD_ANALYTIC, PSD_TABLE, ASD_TABLE = 0, 1, 2
NPAR_SRC, NPAR_MAX = 13, 14


class Events(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("par", ctypes.c_void_p),
                ("tc_s", ctypes.c_void_p), ("active", ctypes.c_void_p), ("par_mask", ctypes.c_void_p),
                ("ecc", ctypes.c_void_p), ("f_ref_ecc", ctypes.c_void_p)]


class SiteDesc(ctypes.Structure):
    _fields_ = [("lat", ctypes.c_double), ("lon", ctypes.c_double), ("gamma", ctypes.c_double),
                ("zeta", ctypes.c_double), ("shape", ctypes.c_int32), ("psd_kind", ctypes.c_int32),
                ("S0", ctypes.c_double), ("f0", ctypes.c_double), ("psd_f", ctypes.c_void_p),
                ("psd_S", ctypes.c_void_p), ("psd_n", ctypes.c_int64)]


class Network(ctypes.Structure):
    _fields_ = [("n_site", ctypes.c_int32), ("site", ctypes.POINTER(SiteDesc))]


class Grid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("fmin", ctypes.c_void_p), ("fmax", ctypes.c_void_p),
                ("npts", ctypes.c_void_p), ("off", ctypes.c_void_p), ("f", ctypes.c_void_p)]


GRID_LOG, GRID_EXPLICIT = 0, 1


class PlanOptions(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("inv_method", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("n_items", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_int64), ("tuned_ms", ctypes.c_double),
                ("items_ms", ctypes.c_double)]


_lib = None


class CovOptions(ctypes.Structure):
    _fields_ = [("fixed_mask", ctypes.c_uint32), ("marg_mask", ctypes.c_uint32),
                ("prior", ctypes.c_double * 14), ("cond_max", ctypes.c_double),
                ("sky_level", ctypes.c_double), ("i_theta", ctypes.c_int32), ("i_phi", ctypes.c_int32),
                ("sky_units", ctypes.c_int32), ("method", ctypes.c_int32), ("truncate", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("svals_thresh", ctypes.c_double), ("par_mask", ctypes.c_void_p)]


SKY_STERAD, SKY_SQDEG = 0, 1
INV_METHODS = {"cho": 0, "cho_svd": 1, "svd": 2, "svd_reg": 3, "cho_dd": 4}


class GwfError(RuntimeError):
    pass


def load():
    """Load libgwf.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise GwfError(f"{LIB_PATH} is missing: build it with `python -m paper_2207_06910_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, d, i32, i64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        lib.gwf_snr.argtypes = [ctypes.POINTER(Events), ctypes.POINTER(Network), ctypes.POINTER(Grid),
                                ctypes.c_uint32, vp, vp, vp, vp]
        lib.gwf_snr.restype = i32
        lib.gwf_fisher.argtypes = [ctypes.POINTER(Events), ctypes.POINTER(Network),
                                   ctypes.POINTER(Grid), ctypes.c_uint32, d, vp, vp, vp, vp, vp]
        lib.gwf_fisher.restype = i32
        lib.gwf_waveform.argtypes = [ctypes.POINTER(Events), ctypes.POINTER(Network),
                                     ctypes.POINTER(Grid), ctypes.c_uint32, vp, i64, vp, vp, vp]
        lib.gwf_waveform.restype = i32
        lib.gwf_fisher_ifo.argtypes = [ctypes.POINTER(Events), ctypes.POINTER(Network),
                                       ctypes.POINTER(Grid), ctypes.c_uint32, vp, vp, vp]
        lib.gwf_fisher_ifo.restype = i32
        lib.gwf_waveform_deriv.argtypes = lib.gwf_waveform.argtypes
        lib.gwf_waveform_deriv.restype = i32
        lib.gwf_invert.argtypes = [i32, i64, vp, d, vp, vp, vp, vp, vp, vp, vp]
        lib.gwf_invert.restype = i32
        lib.gwf_covariance.argtypes = [i32, i64, vp, ctypes.POINTER(CovOptions), vp, vp, vp, vp, vp, vp, vp,
                                       vp, vp, vp, vp]
        lib.gwf_covariance.restype = i32
        lib.gwf_fisher_basis.argtypes = [i32, i64, vp, ctypes.POINTER(Events), ctypes.c_uint32, vp, vp, vp]
        lib.gwf_fisher_basis.restype = i32
        lib.gwf_fisher_adjoint.argtypes = [ctypes.POINTER(Events), ctypes.POINTER(Network),
                                           ctypes.POINTER(Grid), ctypes.c_uint32, vp, vp, d, d,
                                           vp, vp, vp]
        lib.gwf_fisher_adjoint.restype = i32
        lib.gwf_plan_create.argtypes = [ctypes.POINTER(Events), ctypes.POINTER(Network),
                                        ctypes.POINTER(Grid), ctypes.c_uint32,
                                        ctypes.POINTER(PlanOptions), ctypes.POINTER(vp), vp]
        lib.gwf_plan_create.restype = i32
        lib.gwf_plan_fisher.argtypes = [vp, vp, vp, vp, d, vp, vp, vp, vp, vp]
        lib.gwf_plan_fisher.restype = i32
        lib.gwf_fisher_static.argtypes = [ctypes.POINTER(Events), ctypes.POINTER(Network),
                                          ctypes.POINTER(Grid), ctypes.c_uint32, i32, i32, vp, vp, vp, vp]
        lib.gwf_fisher_static.restype = i32
        lib.gwf_plan_adjoint.argtypes = [vp, vp, vp, d, d, vp, vp, vp]
        lib.gwf_plan_adjoint.restype = i32
        lib.gwf_plan_set_network.argtypes = [vp, ctypes.POINTER(Network)]
        lib.gwf_plan_set_network.restype = i32
        lib.gwf_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        lib.gwf_plan_get_info.restype = i32
        lib.gwf_plan_destroy.argtypes = [vp]
        lib.gwf_plan_destroy.restype = i32
        lib.gwf_network_n_ifo.argtypes = [ctypes.POINTER(Network)]
        lib.gwf_network_n_ifo.restype = i32
        lib.gwf_last_error.restype = ctypes.c_char_p
        lib.gwf_version.restype = i32
        _lib = lib
    return _lib


def n_params(flags) -> int:
    """Fisher rows of a call: 11, plus the deformabilities with TIDAL, plus
    e0 with ECCENTRIC."""
    return 11 + (2 if flags & TIDAL else 0) + (1 if flags & ECCENTRIC else 0)


def _check(code, what):
    if code != GWF_OK:
        msg = load().gwf_last_error().decode()
        raise GwfError(f"{what} failed with status {code}: {msg}")


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise GwfError("expected a contiguous float64 tensor on a HIP device")
    return t


def network(sites, curves=None, geometry_only=False) -> tuple:
    """ctypes network descriptor from a list of objects with lat, lon, gamma,
    zeta, shape, S0, f0 attributes (radians, 1/Hz, Hz) and optionally
    psd_kind; ``curves`` holds, per site, None or the (frequencies, values)
    device tensors of its sampled noise curve."""
    arr = (SiteDesc * len(sites))()
    for i, s in enumerate(sites):
        c = None if curves is None else curves[i]
        kind = PSD_ANALYTIC if geometry_only else int(getattr(s, "psd_kind", PSD_ANALYTIC))
        if kind != PSD_ANALYTIC and c is None:
            raise GwfError(f"site {i}: a sampled noise curve needs its device arrays")
        arr[i] = SiteDesc(s.lat, s.lon, s.gamma, s.zeta, int(s.shape), kind, s.S0, s.f0,
                          None if c is None else c[0].data_ptr(), None if c is None else c[1].data_ptr(),
                          0 if c is None else int(c[0].numel()))
    net = Network(len(sites), ctypes.cast(arr, ctypes.POINTER(SiteDesc)))
    return net, arr   # keep arr alive with net


def upload_curves(sites, device="cuda"):
    """Device copies (frequencies, values) of the sites' sampled noise
    curves, None for analytic ones."""
    import torch
    out = []
    for s in sites:
        if int(getattr(s, "psd_kind", PSD_ANALYTIC)) == PSD_ANALYTIC:
            out.append(None)
        else:
            out.append((torch.as_tensor(np.ascontiguousarray(s.psd_f, dtype=np.float64), device=device),
                        torch.as_tensor(np.ascontiguousarray(s.psd_S, dtype=np.float64), device=device)))
    return out


def n_ifo(sites) -> int:
    net, keep = network(sites, geometry_only=True)
    n = load().gwf_network_n_ifo(ctypes.byref(net))
    if n < 0:
        _check(GWF_E_INVALID_ARG, "gwf_network_n_ifo")
    return n


class DeviceWorkload:
    """Device-resident inputs of a synthetic workload (parameters [13][N],
    grid descriptors), plus the host-side network and flags."""

    def __init__(self, wl, device="cuda"):
        import torch
        self.wl = wl
        self.n = wl.n
        self.flags = wl.flags
        self.npar = wl.npar
        self.sites = list(wl.sites)
        self.par = torch.as_tensor(np.ascontiguousarray(wl.par), dtype=torch.float64, device=device)
        self.fmin = torch.as_tensor(np.ascontiguousarray(wl.fmin), dtype=torch.float64, device=device)
        self.fmax = None if wl.fmax is None else torch.as_tensor(
            np.ascontiguousarray(wl.fmax), dtype=torch.float64, device=device)
        self.npts = torch.as_tensor(np.ascontiguousarray(wl.npts), dtype=torch.int32, device=device)
        self.tc_s = None if wl.tc_s is None else torch.as_tensor(
            np.ascontiguousarray(wl.tc_s), dtype=torch.float64, device=device)
        act = getattr(wl, "active", None)
        self.active = None if act is None else torch.as_tensor(
            np.ascontiguousarray(act, dtype=np.uint8), device=device)
        gf = getattr(wl, "grid_f", None)
        self.grid_f = None if gf is None else torch.as_tensor(
            np.ascontiguousarray(gf, dtype=np.float64), device=device)
        self.grid_off = None if gf is None else torch.as_tensor(
            np.ascontiguousarray(wl.grid_offsets(), dtype=np.int64), device=device)
        pm = getattr(wl, "par_mask", None)
        self.par_mask = None if pm is None else torch.as_tensor(
            np.ascontiguousarray(pm, dtype=np.uint32).view(np.int32), device=device)
        ecc = getattr(wl, "ecc", None)
        fre = getattr(wl, "f_ref_ecc", None)
        self.ecc = None if ecc is None else torch.as_tensor(np.ascontiguousarray(ecc, dtype=np.float64),
                                                            device=device)
        self.f_ref_ecc = None if fre is None else torch.as_tensor(np.ascontiguousarray(fre, dtype=np.float64),
                                                                  device=device)
        self.curves = upload_curves(self.sites, device)
        self.n_ifo = n_ifo(self.sites)

    def with_sites(self, sites) -> "DeviceWorkload":
        """The same device arrays with another network of the same shapes
        (sampled noise curves uploaded anew when they changed)."""
        import copy
        if [s.shape for s in sites] != [s.shape for s in self.sites]:
            raise GwfError("with_sites keeps the network's site shapes")
        out = copy.copy(self)
        out.sites = list(sites)
        same = all(getattr(a, "psd_f", None) is getattr(b, "psd_f", None) and
                   getattr(a, "psd_S", None) is getattr(b, "psd_S", None) for a, b in zip(sites, self.sites))
        if not same:
            out.curves = upload_curves(out.sites, self.par.device)
        return out

    def descriptors(self):
        ev = Events(self.n, self.par.shape[1], self.par.data_ptr(),
                    None if self.tc_s is None else self.tc_s.data_ptr(),
                    None if self.active is None else self.active.data_ptr(),
                    None if self.par_mask is None else self.par_mask.data_ptr(),
                    None if self.ecc is None else self.ecc.data_ptr(),
                    None if self.f_ref_ecc is None else self.f_ref_ecc.data_ptr())
        net, keep = network(self.sites, self.curves)
        if self.grid_f is None:
            grid = Grid(GRID_LOG, self.fmin.data_ptr(), None if self.fmax is None else self.fmax.data_ptr(),
                        self.npts.data_ptr(), None, None)
        else:
            grid = Grid(GRID_EXPLICIT, None, None, self.npts.data_ptr(), self.grid_off.data_ptr(),
                        self.grid_f.data_ptr())
        return ev, net, grid, keep


def snr(dw: DeviceWorkload, per_ifo=False, stream=None, out=None):
    import torch
    dev = dw.par.device
    res = out if out is not None else {}
    res.setdefault("snr", torch.empty(dw.n, dtype=torch.float64, device=dev))
    if per_ifo:
        res.setdefault("snr_ifo", torch.empty((dw.n_ifo, dw.n), dtype=torch.float64, device=dev))
    res.setdefault("status", torch.empty(dw.n, dtype=torch.int32, device=dev))
    ev, net, grid, keep = dw.descriptors()
    _check(load().gwf_snr(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid), dw.flags,
                          _ptr(res["snr"]), _ptr(res.get("snr_ifo")), _ptr(res["status"]),
                          _stream(stream)), "gwf_snr")
    return res


def fisher(dw: DeviceWorkload, snr_th=0.0, per_ifo_snr=False, stream=None, out=None):
    """Fisher matrices [P][P][N], SNR [N] and status [N] of every event."""
    import torch
    dev = dw.par.device
    P = n_params(dw.flags)
    res = out if out is not None else {}
    res.setdefault("fisher", torch.empty((P, P, dw.n), dtype=torch.float64, device=dev))
    res.setdefault("snr", torch.empty(dw.n, dtype=torch.float64, device=dev))
    res.setdefault("status", torch.empty(dw.n, dtype=torch.int32, device=dev))
    if per_ifo_snr:
        res.setdefault("snr_ifo", torch.empty((dw.n_ifo, dw.n), dtype=torch.float64, device=dev))
    ev, net, grid, keep = dw.descriptors()
    _check(load().gwf_fisher(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid), dw.flags,
                             float(snr_th), _ptr(res["fisher"]), _ptr(res["snr"]),
                             _ptr(res.get("snr_ifo")), _ptr(res["status"]), _stream(stream)),
           "gwf_fisher")
    return res


def waveform(dw: DeviceWorkload, offsets=None, total=None, mixed=False, stream=None, out=None):
    """Strain h [n_ifo][total] (complex128 on the device) of every event on
    its own grid; event e writes columns offsets[e] .. offsets[e]+npts[e]-1
    (default: the grids packed in event order, total = sum of npts).
    mixed: FP32 amplitude and sin/cos of the reduced phase."""
    import torch
    dev = dw.par.device
    if offsets is None:
        ends = torch.cumsum(dw.npts.to(torch.int64), 0)
        offsets = ends - dw.npts.to(torch.int64)
        if total is None:
            total = int(ends[-1].item())
    if not (offsets.is_cuda and offsets.dtype == torch.int64 and offsets.is_contiguous()
            and offsets.numel() == dw.n):
        raise GwfError("offsets must be a contiguous int64 device tensor of n entries")
    if total is None:
        raise GwfError("total is required with explicit offsets")
    res = out if out is not None else {}
    res.setdefault("h", torch.empty((dw.n_ifo, total), dtype=torch.complex128, device=dev))
    res.setdefault("status", torch.empty(dw.n, dtype=torch.int32, device=dev))
    h = res["h"]
    if not (h.is_cuda and h.dtype == torch.complex128 and h.is_contiguous()
            and tuple(h.shape) == (dw.n_ifo, total)):
        raise GwfError(f"h must be a contiguous complex128 device tensor of shape ({dw.n_ifo}, {total})")
    ev, net, grid, keep = dw.descriptors()
    _check(load().gwf_waveform(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid),
                               dw.flags | (MIXED if mixed else 0),
                               _ptr(offsets), int(total), _ptr(h), _ptr(res["status"]),
                               _stream(stream)), "gwf_waveform")
    return res


def fisher_ifo(dw: DeviceWorkload, stream=None, out=None):
    """Fisher matrix of every interferometer on its own, fisher_ifo
    [n_ifo][P][P][N] (float64 on the device), whose sum over interferometers
    is fisher()'s; plus the parameter status."""
    import torch
    dev = dw.par.device
    P = n_params(dw.flags)
    res = out if out is not None else {}
    res.setdefault("fisher_ifo", torch.empty((dw.n_ifo, P, P, dw.n), dtype=torch.float64, device=dev))
    res.setdefault("status", torch.empty(dw.n, dtype=torch.int32, device=dev))
    F = res["fisher_ifo"]
    if not (F.is_cuda and F.dtype == torch.float64 and F.is_contiguous()
            and tuple(F.shape) == (dw.n_ifo, P, P, dw.n)):
        raise GwfError(f"fisher_ifo must be a contiguous float64 device tensor of shape ({dw.n_ifo}, {P}, {P}, {dw.n})")
    ev, net, grid, keep = dw.descriptors()
    _check(load().gwf_fisher_ifo(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid), dw.flags,
                                 _ptr(F), _ptr(res["status"]), _stream(stream)), "gwf_fisher_ifo")
    return res


def waveform_deriv(dw: DeviceWorkload, offsets=None, total=None, stream=None, out=None):
    """Strain derivatives dh [P][n_ifo][total] (complex128 on the device):
    dh[a, i] is d h_i / d parameter a in the Fisher matrix's rows and units,
    laid out over columns as by waveform(); P = 13 with tides, else 11."""
    import torch
    dev = dw.par.device
    if offsets is None:
        ends = torch.cumsum(dw.npts.to(torch.int64), 0)
        offsets = ends - dw.npts.to(torch.int64)
        if total is None:
            total = int(ends[-1].item())
    if not (offsets.is_cuda and offsets.dtype == torch.int64 and offsets.is_contiguous()
            and offsets.numel() == dw.n):
        raise GwfError("offsets must be a contiguous int64 device tensor of n entries")
    if total is None:
        raise GwfError("total is required with explicit offsets")
    P = n_params(dw.flags)
    res = out if out is not None else {}
    res.setdefault("dh", torch.empty((P, dw.n_ifo, total), dtype=torch.complex128, device=dev))
    res.setdefault("status", torch.empty(dw.n, dtype=torch.int32, device=dev))
    dh = res["dh"]
    if not (dh.is_cuda and dh.dtype == torch.complex128 and dh.is_contiguous()
            and tuple(dh.shape) == (P, dw.n_ifo, total)):
        raise GwfError(f"dh must be a contiguous complex128 device tensor of shape ({P}, {dw.n_ifo}, {total})")
    ev, net, grid, keep = dw.descriptors()
    _check(load().gwf_waveform_deriv(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid), dw.flags,
                                     _ptr(offsets), int(total), _ptr(dh), _ptr(res["status"]),
                                     _stream(stream)), "gwf_waveform_deriv")
    return res


def invert(F, status=None, cond_max=1e50, want_cov=True, par_mask=None, stream=None, out=None):
    """Covariances of Fisher matrices F [P][P][N] (float64, on the device).
    With ``par_mask`` (per-event parameter sets, see covariance) the call
    goes through gwf_covariance with no other manipulation."""
    import torch
    if par_mask is not None:
        res = covariance(F, status, cond_max=cond_max, par_mask=par_mask, want_cov=want_cov,
                         stream=stream, out=out)
        res.pop("out", None)
        return res
    _dev_f64(F)
    P, P2, n = F.shape
    if P != P2:
        raise GwfError("Fisher array must be [P][P][N]")
    dev = F.device
    res = out if out is not None else {}
    if want_cov:
        res.setdefault("cov", torch.empty((P, P, n), dtype=torch.float64, device=dev))
    res.setdefault("sigma", torch.empty((P, n), dtype=torch.float64, device=dev))
    res.setdefault("cond", torch.empty(n, dtype=torch.float64, device=dev))
    res.setdefault("inv_err", torch.empty(n, dtype=torch.float64, device=dev))
    res.setdefault("logdet", torch.empty(n, dtype=torch.float64, device=dev))
    st = status.clone() if status is not None else torch.zeros(n, dtype=torch.int32, device=dev)
    res["status"] = st
    _check(load().gwf_invert(P, n, _ptr(F), float(cond_max), _ptr(res.get("cov")),
                             _ptr(res["sigma"]), _ptr(res["cond"]), _ptr(res["inv_err"]),
                             _ptr(res["logdet"]), _ptr(st), _stream(stream)), "gwf_invert")
    return res


def covariance(F, status=None, fixed=(), prior=None, marg=(), theta=None, sky_level=90.0, units="SqDeg",
               i_theta=3, i_phi=4, cond_max=1e50, method="cho", truncate=False, svals_thresh=1e-15,
               eigen=False, par_mask=None, want_cov=True, stream=None, out=None):
    """Covariances of Fisher matrices F [P][P][N] after the manipulations of
    gwf_covariance: parameters in ``fixed`` held at their fiducial values,
    ``prior`` {index: inverse variance} added before inversion, parameters in
    ``marg`` marginalised over; with ``theta`` [N] (device) the sky area at
    ``sky_level`` percent in ``units`` ("SqDeg" or "Sterad").  Indices refer
    to the P rows of F.  Returns cov [Po][Po][N], sigma [Po][N], cond, inv_err,
    logdet, status, sky (if requested) and ``out``, the indices of F's rows
    in cov and sigma.  ``method``: "cho", "cho_svd", "svd" (with
    ``truncate``), "svd_reg" or "cho_dd" (double-double Cholesky); ``eigen``: also eigval [Pk][N] and eigvec
    [Pk][Pk][N] of the normalised matrix that is inverted; ``par_mask``: a
    device int32 tensor [N] of per-event parameter sets (bit i: row i of F),
    e.g. a DeviceWorkload's ``par_mask``: rows outside an event's set get
    zero covariance rows and columns and a NaN sigma."""
    import torch
    _dev_f64(F)
    P, P2, n = F.shape
    if P != P2:
        raise GwfError("Fisher array must be [P][P][N]")
    o = CovOptions()
    o.fixed_mask = sum(1 << int(i) for i in set(fixed))
    o.marg_mask = sum(1 << int(i) for i in set(marg))
    for i, v in (prior or {}).items():
        o.prior[int(i)] = float(v)
    o.cond_max = float(cond_max)
    o.i_theta, o.i_phi = int(i_theta), int(i_phi)
    o.sky_units = {"SqDeg": SKY_SQDEG, "Sterad": SKY_STERAD}[units]
    o.sky_level = float(sky_level) if theta is not None else 0.0
    o.method = INV_METHODS[method]
    o.truncate = int(bool(truncate))
    o.svals_thresh = float(svals_thresh)
    if par_mask is not None:
        if not (par_mask.is_cuda and par_mask.dtype in (torch.int32, torch.uint32)
                and par_mask.is_contiguous() and par_mask.shape == (n,)):
            raise GwfError("par_mask must be a contiguous int32 tensor [N] on the device")
        o.par_mask = par_mask.data_ptr()
    out_idx = [i for i in range(P) if not (o.fixed_mask >> i & 1) and not (o.marg_mask >> i & 1)]
    po = len(out_idx)
    dev = F.device
    res = out if out is not None else {}
    if want_cov:
        res.setdefault("cov", torch.empty((po, po, n), dtype=torch.float64, device=dev))
    res.setdefault("sigma", torch.empty((po, n), dtype=torch.float64, device=dev))
    for k in ("cond", "inv_err", "logdet"):
        res.setdefault(k, torch.empty(n, dtype=torch.float64, device=dev))
    if theta is not None:
        _dev_f64(theta)
        res.setdefault("sky", torch.empty(n, dtype=torch.float64, device=dev))
    pk = P - len(set(fixed))
    if eigen:
        res.setdefault("eigval", torch.empty((pk, n), dtype=torch.float64, device=dev))
        res.setdefault("eigvec", torch.empty((pk, pk, n), dtype=torch.float64, device=dev))
    st = status.clone() if status is not None else torch.zeros(n, dtype=torch.int32, device=dev)
    res["status"] = st
    _check(load().gwf_covariance(P, n, _ptr(F), ctypes.byref(o), _ptr(theta), _ptr(res.get("cov")),
                                 _ptr(res["sigma"]), _ptr(res["cond"]), _ptr(res["inv_err"]),
                                 _ptr(res["logdet"]), _ptr(res.get("sky")), _ptr(res.get("eigval")),
                                 _ptr(res.get("eigvec")), _ptr(st), _stream(stream)),
           "gwf_covariance")
    res["out"] = out_idx
    return res


BASES = {"chi_sa": 1, "lambda_tilde": 2, "m1m2": 4}


def fisher_basis(F, dw: "DeviceWorkload", basis=("chi_sa", "lambda_tilde"), status=None, out=None, stream=None):
    """The Fisher matrices F [P][P][N] of the workload's events in other
    parameter bases (gwf_fisher_basis): any of "chi_sa", "lambda_tilde",
    "m1m2".  out=F transforms in place."""
    import torch
    _dev_f64(F)
    P, _, n = F.shape
    res = out if out is not None else torch.empty_like(F)
    ev, net, grid, keep = dw.descriptors()
    bits = 0
    for b in basis:
        bits |= BASES[b]
    _check(load().gwf_fisher_basis(P, n, _ptr(F), ctypes.byref(ev), bits, _ptr(res), _ptr(status),
                                   _stream(stream)), "gwf_fisher_basis")
    return res


def fisher_adjoint(dw: DeviceWorkload, gbar, status=None, w_snr=1.0, w_fisher=1.0, stream=None,
                   out=None):
    """Gradient [n_site][4] of sum_e (w_snr ln SNR_e + w_fisher sum_ij gbar_ij Gamma_ij) along
    (latitude, longitude, gamma, ln S0) of every site, gbar [P][P][N] held fixed
    (gbar = Gamma^-1 gives the gradient of sum ln det Gamma); also the per-event
    terms grad_event [N][n_site][4]."""
    import torch
    dev = dw.par.device
    _dev_f64(gbar)
    ns = len(dw.sites)
    res = out if out is not None else {}
    res.setdefault("grad_event", torch.empty((dw.n, ns, 4), dtype=torch.float64, device=dev))
    res.setdefault("grad", torch.empty((ns, 4), dtype=torch.float64, device=dev))
    ev, net, grid, keep = dw.descriptors()
    _check(load().gwf_fisher_adjoint(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid),
                                     dw.flags, _ptr(gbar), _ptr(status), float(w_snr),
                                     float(w_fisher), _ptr(res["grad_event"]), _ptr(res["grad"]),
                                     _stream(stream)), "gwf_fisher_adjoint")
    return res


def fisher_static(dw: DeviceWorkload, chunk=4096, npts_max=None, mixed=False, stream=None, out=None):
    """The batched form without device allocation (gwf_fisher_static): Fisher
    [P][P][N], SNR and status of the workload, the workspace in the library's
    fixed device array.  ``npts_max`` bounds the grid lengths (default: the
    host workload's longest grid)."""
    import torch
    dev = dw.par.device
    P = n_params(dw.flags)
    res = out if out is not None else {}
    res.setdefault("fisher", torch.empty((P, P, dw.n), dtype=torch.float64, device=dev))
    res.setdefault("snr", torch.empty(dw.n, dtype=torch.float64, device=dev))
    res.setdefault("status", torch.empty(dw.n, dtype=torch.int32, device=dev))
    if npts_max is None:
        npts_max = int(np.max(dw.wl.npts))
    ev, net, grid, keep = dw.descriptors()
    _check(load().gwf_fisher_static(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid),
                                    dw.flags | (MIXED if mixed else 0), int(chunk), int(npts_max),
                                    _ptr(res["fisher"]), _ptr(res["snr"]), _ptr(res["status"]),
                                    _stream(stream)), "gwf_fisher_static")
    return res


class Plan:
    """Batched form (gwf_plan_*): built once for a device-resident
    catalogue, then replayed.  Keeps a reference to the DeviceWorkload, whose
    arrays the plan reads at every run."""

    def __init__(self, dw: DeviceWorkload, chunk=0, use_graph=True, profile=False,
                 mixed=False, inv_method="cho", stream=None):
        self.dw = dw
        self.handle = ctypes.c_void_p()
        ev, net, grid, keep = dw.descriptors()
        opt = PlanOptions(int(chunk), 1 if use_graph else 0, 1 if profile else 0, INV_METHODS[inv_method])
        _check(load().gwf_plan_create(ctypes.byref(ev), ctypes.byref(net), ctypes.byref(grid),
                                      dw.flags | (MIXED if mixed else 0), ctypes.byref(opt),
                                      ctypes.byref(self.handle),
                                      _stream(stream)), "gwf_plan_create")
        self.P = n_params(dw.flags)

    def info(self) -> dict:
        i = PlanInfo()
        _check(load().gwf_plan_get_info(self.handle, ctypes.byref(i)), "gwf_plan_get_info")
        return {f: getattr(i, f) for f, _ in PlanInfo._fields_ if f != "pad"}

    def run(self, invert=False, cond_max=1e50, stream=None, out=None):
        import torch
        dev = self.dw.par.device
        n, P = self.dw.n, self.P
        res = out if out is not None else {}
        res.setdefault("fisher", torch.empty((P, P, n), dtype=torch.float64, device=dev))
        res.setdefault("snr", torch.empty(n, dtype=torch.float64, device=dev))
        res.setdefault("status", torch.empty(n, dtype=torch.int32, device=dev))
        if invert:
            res.setdefault("cov", torch.empty((P, P, n), dtype=torch.float64, device=dev))
            res.setdefault("sigma", torch.empty((P, n), dtype=torch.float64, device=dev))
            res.setdefault("cond", torch.empty(n, dtype=torch.float64, device=dev))
            res.setdefault("inv_err", torch.empty(n, dtype=torch.float64, device=dev))
        _check(load().gwf_plan_fisher(self.handle, _ptr(res["fisher"]), _ptr(res["snr"]),
                                      _ptr(res["status"]), float(cond_max), _ptr(res.get("cov")),
                                      _ptr(res.get("sigma")), _ptr(res.get("cond")),
                                      _ptr(res.get("inv_err")), _stream(stream)), "gwf_plan_fisher")
        return res

    def set_sites(self, sites):
        """Replace the plan's network (gwf_plan_set_network), e.g. for a step
        in the detector parameters; sampled noise curves are uploaded."""
        curves = upload_curves(sites, self.dw.par.device)
        net, keep = network(sites, curves)
        _check(load().gwf_plan_set_network(self.handle, ctypes.byref(net)), "gwf_plan_set_network")
        self.sites, self._curves = list(sites), curves

    def adjoint(self, gbar, status=None, w_snr=1.0, w_fisher=1.0, stream=None, out=None):
        """gwf_plan_adjoint: grad [n_site][4] and grad_event [N][n_site][4] of
        sum_e (w_snr ln SNR_e + w_fisher sum_ij gbar_ij Gamma_ij) along every
        site's (latitude, longitude, gamma, ln S0), over the plan's work items."""
        import torch
        _dev_f64(gbar)
        dev = self.dw.par.device
        ns = len(getattr(self, "sites", self.dw.sites))
        res = out if out is not None else {}
        res.setdefault("grad_event", torch.empty((self.dw.n, ns, 4), dtype=torch.float64, device=dev))
        res.setdefault("grad", torch.empty((ns, 4), dtype=torch.float64, device=dev))
        _check(load().gwf_plan_adjoint(self.handle, _ptr(gbar), _ptr(status), float(w_snr), float(w_fisher),
                                       _ptr(res["grad_event"]), _ptr(res["grad"]), _stream(stream)),
               "gwf_plan_adjoint")
        return res

    def close(self):
        if self.handle:
            load().gwf_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

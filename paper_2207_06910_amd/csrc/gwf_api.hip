// gwf_api.hip -- host side of the C ABI declared in include/gwf.h:
// argument validation, network descriptor packing and kernel launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/gwf.h"
#include "gwf_api_internal.hpp"
#include "gwf_kernels.hpp"

namespace {

thread_local std::string g_last_error;

}  // namespace

gwf_status api_fail(gwf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

gwf_status api_hip_fail(hipError_t err, const char* where) {
  return api_fail(GWF_E_HIP, "%s: %s", where, hipGetErrorString(err));
}

namespace {

bool finite_all(std::initializer_list<double> xs) {
  for (double x : xs)
    if (!std::isfinite(x)) return false;
  return true;
}

}  // namespace

// Validate and pack the network into the kernels' by-value descriptor.
gwf_status api_pack_network(const gwf_network* net, gwf::NetDesc& nd) {
  if (!net || !net->site) return api_fail(GWF_E_INVALID_ARG, "network or its site array is NULL");
  if (net->n_site < 1 || net->n_site > GWF_MAX_SITES)
    return api_fail(GWF_E_INVALID_ARG, "n_site=%d outside 1..%d", net->n_site, GWF_MAX_SITES);
  std::memset(&nd, 0, sizeof nd);
  int n_ifo = 0;
  for (int s = 0; s < net->n_site; ++s) {
    const gwf_site& in = net->site[s];
    if (in.shape != GWF_SHAPE_L && in.shape != GWF_SHAPE_T)
      return api_fail(GWF_E_INVALID_ARG, "site %d: shape %d is neither L nor T", s, in.shape);
    if (in.psd_kind != GWF_PSD_ANALYTIC && in.psd_kind != GWF_PSD_TABLE && in.psd_kind != GWF_ASD_TABLE)
      return api_fail(GWF_E_INVALID_ARG, "site %d: psd_kind %d unknown", s, in.psd_kind);
    const bool table = in.psd_kind != GWF_PSD_ANALYTIC;
    if (!finite_all({in.lat, in.lon, in.gamma, in.zeta, in.S0}) || (!table && !std::isfinite(in.f0)))
      return api_fail(GWF_E_INVALID_ARG, "site %d: non-finite geometry or PSD parameter", s);
    if (!(in.S0 > 0.0) || (!table && !(in.f0 > 0.0)))
      return api_fail(GWF_E_INVALID_ARG, "site %d: S0 and f0 must be > 0", s);
    if (table && (!in.psd_f || !in.psd_S || in.psd_n < 2 || in.psd_n > 0x7fffffffLL))
      return api_fail(GWF_E_INVALID_ARG, "site %d: a sampled noise curve needs psd_f, psd_S and 2 <= psd_n < 2^31",
                      s);
    if (std::fabs(in.lat) > 0.5 * M_PI + 1e-12)
      return api_fail(GWF_E_INVALID_ARG, "site %d: latitude outside [-pi/2, pi/2]", s);
    gwf::SiteDesc& o = nd.site[s];
    o.lat = in.lat; o.lon = in.lon; o.gamma = in.gamma; o.zeta = in.zeta;
    o.S0 = in.S0; o.f0 = table ? 1.0 : in.f0; o.shape = in.shape;   // f0 is not read for a sampled curve
    o.psd_kind = in.psd_kind;
    o.tab_f = table ? in.psd_f : nullptr;
    o.tab_S = table ? in.psd_S : nullptr;
    o.tab_n = table ? in.psd_n : 0;
    n_ifo += in.shape == GWF_SHAPE_T ? 3 : 1;
  }
  if (n_ifo > GWF_MAX_IFO) return api_fail(GWF_E_INVALID_ARG, "%d interferometers > %d", n_ifo, GWF_MAX_IFO);
  nd.n_site = net->n_site;
  nd.n_ifo = n_ifo;
  return GWF_OK;
}

gwf_status api_check_common(const gwf_events* ev, const gwf_grid* grid, uint32_t flags) {
  if (!ev || !grid) return api_fail(GWF_E_INVALID_ARG, "events or grid descriptor is NULL");
  if (ev->n < 1) return api_fail(GWF_E_INVALID_ARG, "n=%lld must be >= 1", (long long)ev->n);
  if (ev->n > 0x7fffffffLL) return api_fail(GWF_E_INVALID_ARG, "n=%lld exceeds 2^31-1", (long long)ev->n);
  if (ev->ld < ev->n) return api_fail(GWF_E_INVALID_ARG, "ld=%lld < n", (long long)ev->ld);
  if (!ev->par) return api_fail(GWF_E_INVALID_ARG, "par is NULL");
  if (grid->kind == GWF_GRID_LOG) {
    if (!grid->fmin || !grid->npts) return api_fail(GWF_E_INVALID_ARG, "grid fmin or npts is NULL");
  } else if (grid->kind == GWF_GRID_EXPLICIT) {
    if (!grid->off || !grid->f || !grid->npts)
      return api_fail(GWF_E_INVALID_ARG, "explicit grid off, f or npts is NULL");
  } else {
    return api_fail(GWF_E_UNSUPPORTED, "grid kind %d", grid->kind);
  }
  if (flags & ~(uint32_t)(GWF_EARTH_ROT | GWF_TIDAL | GWF_MIXED | GWF_ECCENTRIC))
    return api_fail(GWF_E_INVALID_ARG, "unknown flag bits 0x%x", flags);
  if ((flags & GWF_ECCENTRIC) && !ev->ecc) return api_fail(GWF_E_INVALID_ARG, "GWF_ECCENTRIC needs ev->ecc");
  return GWF_OK;
}

// The explicit grid's offsets and frequencies, or NULLs for a log grid.
inline void api_explicit_grid(const gwf_grid* grid, const int64_t*& off, const double*& f) {
  const bool ex = grid->kind == GWF_GRID_EXPLICIT;
  off = ex ? grid->off : nullptr;
  f = ex ? grid->f : nullptr;
}

extern "C" {

const char* gwf_last_error(void) { return g_last_error.c_str(); }

int32_t gwf_version(void) { return GWF_VERSION; }

int32_t gwf_network_n_ifo(const gwf_network* net) {
  gwf::NetDesc nd;
  if (api_pack_network(net, nd) != GWF_OK) return -1;
  return nd.n_ifo;
}

gwf_status gwf_snr(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                   uint32_t flags, double* snr, double* snr_ifo, int32_t* status, void* stream) {
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (!snr) return api_fail(GWF_E_INVALID_ARG, "snr is NULL");
  if (flags & GWF_MIXED) return api_fail(GWF_E_UNSUPPORTED, "the mixed form runs through a plan");
  gwf::SnrArgs a{};
  if ((st = api_pack_network(net, a.net))) return st;
  a.par = ev->par; a.ld = ev->ld; a.n = ev->n;
  a.fmin = grid->fmin; a.fmax = grid->fmax; a.npts = grid->npts;
  api_explicit_grid(grid, a.goff, a.gf);
  a.tidal = (flags & GWF_TIDAL) ? 1 : 0;
  a.active = ev->active;
  a.snr = snr; a.snr_ifo = snr_ifo; a.status = status;
  hipError_t err = gwf::launch_snr(a, (flags & GWF_EARTH_ROT) != 0, (hipStream_t)stream);
  if (err != hipSuccess) return api_hip_fail(err, "snr kernel launch");
  return GWF_OK;
}

gwf_status gwf_fisher(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                      uint32_t flags, double snr_th, double* fisher, double* snr, double* snr_ifo,
                      int32_t* status, void* stream) {
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (!fisher || !snr || !status) return api_fail(GWF_E_INVALID_ARG, "fisher, snr and status are required");
  if (!std::isfinite(snr_th)) return api_fail(GWF_E_INVALID_ARG, "snr_th is not finite");
  if (flags & GWF_MIXED) return api_fail(GWF_E_UNSUPPORTED, "the mixed form runs through a plan");
  gwf::FisherArgs a{};
  if ((st = api_pack_network(net, a.net))) return st;
  a.par = ev->par; a.ld = ev->ld; a.n = ev->n;
  a.fmin = grid->fmin; a.fmax = grid->fmax; a.npts = grid->npts;
  api_explicit_grid(grid, a.goff, a.gf);
  a.snr_th = snr_th;
  a.active = ev->active;
  a.par_mask = ev->par_mask;
  a.fisher = fisher; a.snr = snr; a.status = status;
  const bool rot = (flags & GWF_EARTH_ROT) != 0, tidal = (flags & GWF_TIDAL) != 0;
  a.ecc = ev->ecc; a.fref = ev->f_ref_ecc;
  hipStream_t s = (hipStream_t)stream;
  // per-interferometer SNRs, or the SNR pass that decides the threshold
  if (snr_ifo || snr_th > 0.0) {
    gwf::SnrArgs b{};
    b.net = a.net; b.par = a.par; b.ld = a.ld; b.n = a.n;
    b.fmin = a.fmin; b.fmax = a.fmax; b.npts = a.npts; b.tidal = tidal; b.active = a.active;
    b.goff = a.goff; b.gf = a.gf;
    b.snr = snr; b.snr_ifo = snr_ifo; b.status = nullptr;
    hipError_t err = gwf::launch_snr(b, rot, s);
    if (err != hipSuccess) return api_hip_fail(err, "snr kernel launch");
    if (snr_th > 0.0) a.snr_pre = snr;
  }
  hipError_t err = gwf::launch_fisher(a, api_npi(flags), rot, s);
  if (err != hipSuccess) return api_hip_fail(err, "fisher kernel launch");
  return GWF_OK;
}

gwf_status gwf_fisher_ifo(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                          uint32_t flags, double* fisher_ifo, int32_t* status, void* stream) {
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (!fisher_ifo || !status) return api_fail(GWF_E_INVALID_ARG, "fisher_ifo and status are required");
  if (flags & GWF_MIXED) return api_fail(GWF_E_UNSUPPORTED, "the mixed form runs through a plan");
  gwf::FisherArgs a{};
  if ((st = api_pack_network(net, a.net))) return st;
  a.par = ev->par; a.ld = ev->ld; a.n = ev->n;
  a.fmin = grid->fmin; a.fmax = grid->fmax; a.npts = grid->npts;
  api_explicit_grid(grid, a.goff, a.gf);
  a.active = ev->active;
  a.par_mask = ev->par_mask;
  a.snr = nullptr; a.status = status;
  const bool rot = (flags & GWF_EARTH_ROT) != 0;
  const int64_t P = 8 + api_npi(flags);
  a.ecc = ev->ecc; a.fref = ev->f_ref_ecc;
  for (int d = 0; d < a.net.n_ifo; ++d) {
    a.ifo_sel = d + 1;
    a.fisher = fisher_ifo + (int64_t)d * P * P * ev->n;
    hipError_t err = gwf::launch_fisher(a, api_npi(flags), rot, (hipStream_t)stream);
    if (err != hipSuccess) return api_hip_fail(err, "fisher kernel launch");
  }
  return GWF_OK;
}

gwf_status gwf_waveform(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                        uint32_t flags, const int64_t* offsets, int64_t total, double* h,
                        int32_t* status, void* stream) {
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (!offsets || !h) return api_fail(GWF_E_INVALID_ARG, "offsets and h are required");
  if (total < 1) return api_fail(GWF_E_INVALID_ARG, "total=%lld must be >= 1", (long long)total);
  gwf::WaveformArgs a{};
  if ((st = api_pack_network(net, a.net))) return st;
  a.par = ev->par; a.ld = ev->ld; a.n = ev->n; a.tc_s = ev->tc_s;
  a.fmin = grid->fmin; a.fmax = grid->fmax; a.npts = grid->npts;
  api_explicit_grid(grid, a.goff, a.gf);
  a.offsets = offsets; a.total = total; a.h = h; a.status = status;
  a.ecc = ev->ecc; a.fref = ev->f_ref_ecc; a.ecc_flag = flags & GWF_ECCENTRIC;
  hipError_t err = gwf::launch_waveform(a, (flags & GWF_TIDAL) != 0, (flags & GWF_EARTH_ROT) != 0,
                                        (flags & GWF_MIXED) != 0, (hipStream_t)stream);
  if (err != hipSuccess) return api_hip_fail(err, "waveform kernel launch");
  return GWF_OK;
}

gwf_status gwf_waveform_deriv(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                              uint32_t flags, const int64_t* offsets, int64_t total, double* dh,
                              int32_t* status, void* stream) {
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (!offsets || !dh) return api_fail(GWF_E_INVALID_ARG, "offsets and dh are required");
  if (total < 1) return api_fail(GWF_E_INVALID_ARG, "total=%lld must be >= 1", (long long)total);
  if (flags & GWF_MIXED) return api_fail(GWF_E_UNSUPPORTED, "the strain derivatives have no mixed form");
  gwf::WaveformArgs a{};
  if ((st = api_pack_network(net, a.net))) return st;
  a.par = ev->par; a.ld = ev->ld; a.n = ev->n; a.tc_s = ev->tc_s;
  a.fmin = grid->fmin; a.fmax = grid->fmax; a.npts = grid->npts;
  api_explicit_grid(grid, a.goff, a.gf);
  a.offsets = offsets; a.total = total; a.dh = dh; a.status = status; a.par_mask = ev->par_mask;
  a.ecc = ev->ecc; a.fref = ev->f_ref_ecc; a.ecc_flag = flags & GWF_ECCENTRIC;
  hipError_t err = gwf::launch_waveform_deriv(a, api_npi(flags), (flags & GWF_EARTH_ROT) != 0,
                                              (hipStream_t)stream);
  if (err != hipSuccess) return api_hip_fail(err, "waveform derivative kernel launch");
  return GWF_OK;
}

gwf_status gwf_fisher_adjoint(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                              uint32_t flags, const double* gbar, const int32_t* status,
                              double w_snr, double w_fisher, double* grad_event, double* grad,
                              void* stream) {
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (flags & GWF_MIXED) return api_fail(GWF_E_UNSUPPORTED, "the adjoint has no mixed form");
  if (grid->kind == GWF_GRID_EXPLICIT) return api_fail(GWF_E_UNSUPPORTED, "the adjoint needs log grids");
  if (!gbar || !grad_event || !grad) return api_fail(GWF_E_INVALID_ARG, "gbar, grad_event and grad are required");
  if (!std::isfinite(w_snr) || !std::isfinite(w_fisher))
    return api_fail(GWF_E_INVALID_ARG, "w_snr and w_fisher must be finite");
  gwf::AdjointArgs a{};
  if ((st = api_pack_network(net, a.net))) return st;
  a.par = ev->par; a.ld = ev->ld; a.n = ev->n;
  a.fmin = grid->fmin; a.fmax = grid->fmax; a.npts = grid->npts;
  a.gbar = gbar; a.status = status; a.w_snr = w_snr; a.w_fisher = w_fisher;
  a.active = ev->active;
  a.par_mask = ev->par_mask;
  a.grad_event = grad_event; a.grad = grad;
  a.ecc = ev->ecc; a.fref = ev->f_ref_ecc;
  hipError_t err = gwf::launch_adjoint(a, api_npi(flags), (flags & GWF_EARTH_ROT) != 0,
                                       (hipStream_t)stream);
  if (err != hipSuccess) return api_hip_fail(err, "adjoint kernel launch");
  return GWF_OK;
}

gwf_status gwf_invert(int32_t P, int64_t n, const double* fisher, double cond_max, double* cov,
                      double* sigma, double* cond, double* inv_err, double* logdet, int32_t* status,
                      void* stream) {
  if (P < 1 || P > GWF_NPAR_MAX) return api_fail(GWF_E_INVALID_ARG, "P=%d outside 1..%d", P, GWF_NPAR_MAX);
  if (n < 1) return api_fail(GWF_E_INVALID_ARG, "n=%lld must be >= 1", (long long)n);
  if (!fisher || !sigma || !status) return api_fail(GWF_E_INVALID_ARG, "fisher, sigma and status are required");
  if (std::isnan(cond_max)) return api_fail(GWF_E_INVALID_ARG, "cond_max is NaN");
  gwf::InvertArgs a{};
  a.n = n; a.fisher = fisher; a.cond_max = cond_max; a.cov = cov; a.sigma = sigma;
  a.cond = cond; a.inv_err = inv_err; a.logdet = logdet; a.status = status;
  hipError_t err = gwf::launch_invert(a, P, (hipStream_t)stream);
  if (err != hipSuccess) return api_hip_fail(err, "invert kernel launch");
  return GWF_OK;
}

gwf_status gwf_fisher_basis(int32_t P, int64_t n, const double* fisher, const gwf_events* ev,
                            uint32_t basis, double* out, int32_t* status, void* stream) {
  if (P < 11 || P > 14) return api_fail(GWF_E_INVALID_ARG, "P=%d must be 11 to 14", P);
  if (n < 1) return api_fail(GWF_E_INVALID_ARG, "n=%lld must be >= 1", (long long)n);
  if (!fisher || !out || !ev || !ev->par) return api_fail(GWF_E_INVALID_ARG, "fisher, out and ev->par are required");
  if (ev->n != n || ev->ld < n) return api_fail(GWF_E_INVALID_ARG, "ev->n must be n and ev->ld >= n");
  if (basis & ~7u) return api_fail(GWF_E_INVALID_ARG, "basis=%u has unknown bits", basis);
  if ((basis & GWF_BASIS_LAMBDA_TILDE) && P < 13)
    return api_fail(GWF_E_INVALID_ARG, "the tidal basis needs P=13 (or 14 with e0)");
  gwf::BasisArgs a{};
  a.n = n; a.fisher = fisher; a.out = out; a.par = ev->par; a.ld = ev->ld; a.basis = basis; a.status = status;
  hipError_t err = gwf::launch_basis(a, P, (hipStream_t)stream);
  if (err != hipSuccess) return api_hip_fail(err, "basis kernel launch");
  return GWF_OK;
}

gwf_status gwf_covariance(int32_t P, int64_t n, const double* fisher, const gwf_cov_opts* opts,
                          const double* theta, double* cov, double* sigma, double* cond,
                          double* inv_err, double* logdet, double* sky, double* eigval,
                          double* eigvec, int32_t* status, void* stream) {
  if (P < 1 || P > GWF_NPAR_MAX) return api_fail(GWF_E_INVALID_ARG, "P=%d outside 1..%d", P, GWF_NPAR_MAX);
  if (n < 1) return api_fail(GWF_E_INVALID_ARG, "n=%lld must be >= 1", (long long)n);
  if (!fisher || !sigma || !status || !opts)
    return api_fail(GWF_E_INVALID_ARG, "fisher, opts, sigma and status are required");
  const gwf_cov_opts& o = *opts;
  const uint32_t all = (1u << P) - 1u;
  if ((o.fixed_mask & ~all) || (o.marg_mask & ~all))
    return api_fail(GWF_E_INVALID_ARG, "masks name parameters beyond P=%d", P);
  if (o.fixed_mask & o.marg_mask)
    return api_fail(GWF_E_INVALID_ARG, "a parameter cannot be both fixed and marginalised");
  if (std::isnan(o.cond_max)) return api_fail(GWF_E_INVALID_ARG, "cond_max is NaN");
  if (o.method < GWF_INV_CHO || o.method > GWF_INV_CHO_DD)
    return api_fail(GWF_E_INVALID_ARG, "method=%d unknown", o.method);
  if ((o.method == GWF_INV_SVD || o.method == GWF_INV_SVD_REG) &&
      !(o.svals_thresh >= 0.0 && o.svals_thresh < 1.0))
    return api_fail(GWF_E_INVALID_ARG, "svals_thresh=%g must be in [0, 1)", o.svals_thresh);
  gwf::InvertArgs a{};
  a.method = o.method;
  a.truncate = o.truncate != 0;
  a.svals_thresh = (o.method == GWF_INV_SVD || o.method == GWF_INV_SVD_REG) ? o.svals_thresh : 0.0;
  a.eigval = eigval;
  a.eigvec = eigvec;
  a.par_mask = o.par_mask;
  a.n = n; a.fisher = fisher; a.cond_max = o.cond_max; a.cov = cov; a.sigma = sigma;
  a.cond = cond; a.inv_err = inv_err; a.logdet = logdet; a.status = status;
  a.p_full = P;
  int pk = 0, po = 0;
  for (int i = 0; i < GWF_NPAR_MAX; ++i) { a.keep[i] = 0; a.out_pos[i] = -1; a.prior[i] = 0.0; }
  a.i_theta = a.i_phi = -1;
  for (int i = 0; i < P; ++i) {
    if (o.fixed_mask >> i & 1u) continue;
    if (!(o.prior[i] >= 0.0) || !std::isfinite(o.prior[i]))
      return api_fail(GWF_E_INVALID_ARG, "prior[%d]=%g must be finite and >= 0", i, o.prior[i]);
    a.keep[pk] = (int8_t)i;
    a.prior[pk] = o.prior[i];
    if (!(o.marg_mask >> i & 1u)) a.out_pos[pk] = (int8_t)po++;
    if (i == o.i_theta) a.i_theta = pk;
    if (i == o.i_phi) a.i_phi = pk;
    ++pk;
  }
  for (int i = P; i < GWF_NPAR_MAX; ++i)
    if (o.prior[i] != 0.0) return api_fail(GWF_E_INVALID_ARG, "prior[%d] set beyond P=%d", i, P);
  if (po < 1) return api_fail(GWF_E_INVALID_ARG, "no parameter is left after fixing and marginalising");
  a.n_out = po;
  if (o.sky_level > 0.0) {
    if (!(o.sky_level < 100.0)) return api_fail(GWF_E_INVALID_ARG, "sky_level=%g must be below 100", o.sky_level);
    if (!theta || !sky) return api_fail(GWF_E_INVALID_ARG, "theta and sky are required for the sky area");
    if (o.i_theta < 0 || o.i_theta >= P || o.i_phi < 0 || o.i_phi >= P || o.i_theta == o.i_phi)
      return api_fail(GWF_E_INVALID_ARG, "i_theta=%d, i_phi=%d must be distinct indices below P", o.i_theta,
                      o.i_phi);
    if (a.i_theta < 0 || a.i_phi < 0) return api_fail(GWF_E_INVALID_ARG, "theta or phi is fixed");
    if (o.sky_units != GWF_SKY_STERAD && o.sky_units != GWF_SKY_SQDEG)
      return api_fail(GWF_E_INVALID_ARG, "sky_units=%d unknown", o.sky_units);
    const double deg = 180.0 / 3.14159265358979323846;
    a.sky_fac = -2.0 * 3.14159265358979323846 * std::log1p(-o.sky_level / 100.0) *
                (o.sky_units == GWF_SKY_SQDEG ? deg * deg : 1.0);
    a.theta = theta;
    a.sky = sky;
  } else {
    a.i_theta = a.i_phi = -1;
    a.sky = nullptr;
  }
  hipError_t err = gwf::launch_invert(a, pk, (hipStream_t)stream);
  if (err != hipSuccess) return api_hip_fail(err, "covariance kernel launch");
  return GWF_OK;
}

}  // extern "C"

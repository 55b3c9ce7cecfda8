// model_host.hip -- TEST ONLY: the per-point mathematics of the GPU kernels
// (gwf_model.hpp, the same source the kernels compile) run on the host, so
// that the CPU test-suite can compare the kernel math with the oracle
// without a GPU.  Never linked into libgwf; no product path calls it.
#include <cmath>
#include <vector>

#include "../../paper_2207_06910_amd/csrc/gwf_dd.hpp"
#include "../../paper_2207_06910_amd/csrc/gwf_invert.hpp"
#include "../../paper_2207_06910_amd/csrc/gwf_model.hpp"

using namespace gwf;

template <bool TIDAL, bool ROT, bool MIXED>
static void one_event(const double* p, double fmin, double fmax, int32_t n, const NetDesc& nd,
                      double* F, double* snr, int32_t* status) {
  constexpr int P = TIDAL ? 13 : 11, NPI = P - 8, NACC = 36 + 8 * NPI + NPI * (NPI + 1) / 2;
  static_assert(NPI == 3 || NPI == 5, "the host build covers the non-eccentric forms");
  const uint32_t flags = (TIDAL ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u);
  EventC ec;
  event_setup(p, fmin, fmax, n, flags, ec);
  *status = ec.status;
  if (ec.status) return;
  SiteC sc[kMaxSites];
  for (int s = 0; s < nd.n_site; ++s) site_setup(p, nd.site[s], ec, sc[s]);
  double Gacc[kGramAcc] = {0}, G[36], xy[64] = {0};
  for (int32_t k = 0; k < ec.n; ++k) {
    double U[8], W, c[5];
    accumulate_point<NPI, ROT, MIXED>(ec, sc, nd.n_site, k, Gacc, U, W, c);
    add_phase_blocks(NPI, U, W, c, xy, 1);
  }
  gram_finish(ec, Gacc, G);
  for (int t = 0; t < NACC; ++t) {
    int r, c;
    slot_position(t, NPI, r, c);
    const double v = t < 36 ? G[t] : xy[t - 36];
    F[r * P + c] = v;
    F[c * P + r] = v;
  }
  *snr = std::sqrt(F[8 * P + 8]);
}

extern "C" int model_fisher_host(int64_t n, const double* par, int64_t ld, const double* fmin,
                                 const double* fmax, const int32_t* npts, int n_site,
                                 const double* sites, uint32_t flags, double* fisher, double* snr,
                                 int32_t* status) {
  NetDesc nd{};
  nd.n_site = n_site;
  for (int s = 0; s < n_site; ++s) {
    const double* r = sites + 7 * s;
    nd.site[s] = SiteDesc{r[0], r[1], r[2], r[3], r[5], r[6], (int32_t)r[4], 0};
  }
  const bool tidal = flags & kFlagTidal, rot = flags & kFlagRot;
  const int P = tidal ? 13 : 11;
  std::vector<double> F(P * P);
  for (int64_t e = 0; e < n; ++e) {
    double p[kNparIn] = {};
    for (int r = 0; r < 13; ++r) p[r] = par[r * ld + e];
    const double fx = fmax ? fmax[e] : 0.0;
    if (flags & kFlagMixed) {
      if (tidal && rot) one_event<true, true, true>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
      else if (tidal) one_event<true, false, true>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
      else if (rot) one_event<false, true, true>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
      else one_event<false, false, true>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
    } else {
      if (tidal && rot) one_event<true, true, false>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
      else if (tidal) one_event<true, false, false>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
      else if (rot) one_event<false, true, false>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
      else one_event<false, false, false>(p, fmin[e], fx, npts[e], nd, F.data(), snr + e, status + e);
    }
    for (int i = 0; i < P * P; ++i) fisher[i * n + e] = status[e] ? 0.0 : F[i];
  }
  return 0;
}

// Host build of the adjoint's per-point mathematics (gwf_adjoint.hpp): the
// per-event gradient terms grad_event[e][s][m] for a given gbar [P][P][n].
#include "../../paper_2207_06910_amd/csrc/gwf_adjoint.hpp"

template <bool TIDAL, bool ROT>
static void one_event_adjoint(const double* p, double fmin, double fmax, int32_t n, const NetDesc& nd,
                              const double* Gb, double w_snr, double w_fisher, double* ge) {
  const uint32_t flags = (TIDAL ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u);
  constexpr int NPI = TIDAL ? 5 : 3, P = 8 + NPI;
  EventC ec;
  event_setup(p, fmin, fmax, n, flags, ec);
  for (int i = 0; i < nd.n_site * 4; ++i) ge[i] = 0.0;
  if (ec.status) return;
  AdjEventC ae;
  adj_event_setup<NPI>(ec, [&](int i, int j) { return Gb[i * P + j]; }, ae);
  double acc[kMaxSites][kAdjN] = {};
  for (int s = 0; s < nd.n_site; ++s) {
    SiteC sc;
    AdjSiteC as;
    site_setup(p, nd.site[s], ec, sc);
    adj_site_setup(p, nd.site[s], sc, as);
    for (int32_t k = 0; k < ec.n; ++k) adjoint_point<NPI, ROT>(ec, ae, sc, as, k, acc[s]);
  }
  double W = 0.0;
  for (int s = 0; s < nd.n_site; ++s) W += acc[s][kAdjW];
  for (int s = 0; s < nd.n_site; ++s)
    for (int m = 0; m < 4; ++m) {
      const double dS = m < 3 ? acc[s][kAdjS + m] : -acc[s][kAdjW];
      ge[s * 4 + m] = w_fisher * acc[s][kAdjT + m] + w_snr * dS / (2.0 * W);
    }
}

extern "C" int model_adjoint_host(int64_t n, const double* par, int64_t ld, const double* fmin,
                                  const double* fmax, const int32_t* npts, int n_site,
                                  const double* sites, uint32_t flags, const double* gbar,
                                  double w_snr, double w_fisher, double* grad_event) {
  NetDesc nd{};
  nd.n_site = n_site;
  for (int s = 0; s < n_site; ++s) {
    const double* r = sites + 7 * s;
    nd.site[s] = SiteDesc{r[0], r[1], r[2], r[3], r[5], r[6], (int32_t)r[4], 0};
  }
  const bool tidal = flags & kFlagTidal, rot = flags & kFlagRot;
  const int P = tidal ? 13 : 11;
  std::vector<double> G(P * P);
  for (int64_t e = 0; e < n; ++e) {
    double p[kNparIn] = {};
    for (int r = 0; r < 13; ++r) p[r] = par[r * ld + e];
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j)
        G[i * P + j] = 0.5 * (gbar[(i * P + j) * n + e] + gbar[(j * P + i) * n + e]);
    const double fx = fmax ? fmax[e] : 0.0;
    double* ge = grad_event + e * n_site * 4;
    if (tidal && rot) one_event_adjoint<true, true>(p, fmin[e], fx, npts[e], nd, G.data(), w_snr, w_fisher, ge);
    else if (tidal) one_event_adjoint<true, false>(p, fmin[e], fx, npts[e], nd, G.data(), w_snr, w_fisher, ge);
    else if (rot) one_event_adjoint<false, true>(p, fmin[e], fx, npts[e], nd, G.data(), w_snr, w_fisher, ge);
    else one_event_adjoint<false, false>(p, fmin[e], fx, npts[e], nd, G.data(), w_snr, w_fisher, ge);
  }
  return 0;
}

// ---- condition number by the inversion kernel's one-sided Jacobi: lane j
// of the kernel is column j here; every step reads all partner columns
// before any column is rotated, as the lanes' permutes do.
extern "C" int model_jacobi_partner(int M, int j, int t) {
  switch (M) {
    case 2: return jacobi_partner<2>(j, t);
    case 4: return jacobi_partner<4>(j, t);
    case 6: return jacobi_partner<6>(j, t);
    case 8: return jacobi_partner<8>(j, t);
    case 10: return jacobi_partner<10>(j, t);
    case 12: return jacobi_partner<12>(j, t);
    case 14: return jacobi_partner<14>(j, t);
    default: return -1;
  }
}

template <int P>
static void jacobi_cond_one(const double* F, int64_t n, int64_t e, double* cond, int32_t* sweeps) {
  constexpr int M = P + (P & 1), G = 16;
  double x[G][P] = {}, y[G][P];
  double d[P];
  bool normalise = true;
  for (int i = 0; i < P; ++i) normalise = normalise && F[(i * P + i) * n + e] > 0.0;
  for (int i = 0; i < P; ++i) d[i] = normalise ? std::sqrt(F[(i * P + i) * n + e]) : 1.0;
  for (int j = 0; j < P; ++j)
    for (int i = 0; i < P; ++i) {
      const int r = i <= j ? i : j, c = i <= j ? j : i;
      x[j][i] = F[(r * P + c) * n + e] / (d[i] * d[j]);
    }
  int sw = 0;
  for (; sw < 40; ++sw) {
    bool any = false;
    double nrm[G];
    for (int j = 0; j < G; ++j) nrm[j] = col_dot<P>(x[j], x[j]);
    for (int t = 0; t < M - 1; ++t) {
      double ny[G];
      for (int j = 0; j < G; ++j) {
        const int q = jacobi_partner<M>(j, t);
        for (int i = 0; i < P; ++i) y[j][i] = x[q][i];
        ny[j] = nrm[q];
      }
      for (int j = 0; j < G; ++j) {
        const int q = jacobi_partner<M>(j, t);
        if (jacobi_update<P>(x[j], y[j], nrm[j], ny[j], j, q)) any = true;
      }
    }
    if (!any) break;
  }
  double smax = 0.0, smin = INFINITY;
  for (int j = 0; j < P; ++j) {
    const double sv = std::sqrt(col_dot<P>(x[j], x[j]));
    smax = std::fmax(smax, sv);
    smin = std::fmin(smin, sv);
  }
  cond[e] = smin > 0.0 ? smax / smin : INFINITY;
  sweeps[e] = sw + 1;
}

extern "C" int model_jacobi_cond_host(int P, int64_t n, const double* F, double* cond, int32_t* sweeps) {
  for (int64_t e = 0; e < n; ++e) {
    switch (P) {
      case 2: jacobi_cond_one<2>(F, n, e, cond, sweeps); break;
      case 5: jacobi_cond_one<5>(F, n, e, cond, sweeps); break;
      case 9: jacobi_cond_one<9>(F, n, e, cond, sweeps); break;
      case 11: jacobi_cond_one<11>(F, n, e, cond, sweeps); break;
      case 13: jacobi_cond_one<13>(F, n, e, cond, sweeps); break;
      default: return -1;
    }
  }
  return 0;
}

// ---- double-double primitives of the inversion (op: 0 add, 1 sub, 2 mul,
// 3 mul with the operands swapped, 4 div, 5 sqrt of a)
extern "C" void model_dd(int op, const double* a, const double* b, double* out) {
  const dd x{a[0], a[1]}, y{b[0], b[1]};
  dd r{0.0, 0.0};
  switch (op) {
    case 0: r = dd_add(x, y); break;
    case 1: r = dd_sub(x, y); break;
    case 2: r = dd_mul(x, y); break;
    case 3: r = dd_mul(y, x); break;
    case 4: r = dd_div(x, y); break;
    default: r = dd_sqrt(x); break;
  }
  out[0] = r.hi;
  out[1] = r.lo;
}

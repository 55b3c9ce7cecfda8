// gwf_adjoint.hpp -- per-point mathematics of the adjoint of the Fisher/SNR
// map with respect to the detector parameters (latitude, longitude, arm angle
// gamma and ln S0 of each site).
//
// For a figure of merit J(Gamma_e, SNR_e) the reverse-mode sensitivity
// along a detector parameter xi is
//   dJ/dxi = sum_e [ sum_ij Gbar_e,ij dGamma_e,ij/dxi + snrbar_e dSNR_e/dxi ],
// Gbar = dJ/dGamma (Gamma^-1 for J = ln det Gamma), snrbar = dJ/dSNR.  With
// Gamma_ij = sum_{k,d} w Re(D_i D_j^*) (sec. 3.2, D the noise-weighted
// derivative vectors of the phase-free form) and a symmetric Gbar,
//   sum_ij Gbar_ij dGamma_ij = sum_{k,d} [ dw Re(D^H z) + 2 w Re(dD . z^*) ],
//   z = Gbar D,
// so the backward pass recomputes D at every grid point, forms z, and
// contracts it with the derivative of D along each detector parameter; no
// Jacobian is stored.  The derivatives along latitude, longitude and gamma
// are carried by the three-component tangent numbers T3 through the site's
// geometry (patterns, hour angle, arrival-time offset); along ln S0 only the
// weight changes, dw = -w, which gives -sum w Re(D^H z) in closed form.
#pragma once

#include "gwf_model.hpp"

namespace gwf {

// ------------------------------------------------------------- tangents
// A value and its derivatives along (latitude, longitude, gamma) of one site.
struct T3 {
  double v, d[3];
};

__host__ __device__ inline T3 t3c(double v) { return T3{v, {0.0, 0.0, 0.0}}; }
__host__ __device__ inline T3 operator+(const T3& a, const T3& b) {
  return T3{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}};
}
__host__ __device__ inline T3 operator-(const T3& a, const T3& b) {
  return T3{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}};
}
__host__ __device__ inline T3 operator-(const T3& a) { return T3{-a.v, {-a.d[0], -a.d[1], -a.d[2]}}; }
__host__ __device__ inline T3 operator*(const T3& a, const T3& b) {
  return T3{a.v * b.v, {fma(a.d[0], b.v, a.v * b.d[0]), fma(a.d[1], b.v, a.v * b.d[1]),
                        fma(a.d[2], b.v, a.v * b.d[2])}};
}
__host__ __device__ inline T3 operator*(double s, const T3& a) {
  return T3{s * a.v, {s * a.d[0], s * a.d[1], s * a.d[2]}};
}
__host__ __device__ inline T3 operator*(const T3& a, double s) { return s * a; }
__host__ __device__ inline T3 operator+(const T3& a, double s) { return T3{a.v + s, {a.d[0], a.d[1], a.d[2]}}; }
// a * b + c
__host__ __device__ inline T3 fmat(const T3& a, const T3& b, const T3& c) {
  return T3{fma(a.v, b.v, c.v), {fma(a.d[0], b.v, fma(a.v, b.d[0], c.d[0])),
                                 fma(a.d[1], b.v, fma(a.v, b.d[1], c.d[1])),
                                 fma(a.d[2], b.v, fma(a.v, b.d[2], c.d[2]))}};
}
__host__ __device__ inline T3 dot4t(const T3 a[4], const T3 b[4]) {
  return fmat(a[0], b[0], fmat(a[1], b[1], fmat(a[2], b[2], a[3] * b[3])));
}

// ----------------------------------------------------- site constants
// The per-(event, site) constants of site_setup with their derivatives
// along latitude (d[0]), longitude (d[1]) and gamma (d[2]).
struct SiteA {
  T3 cdl, sdl, sl, cl, slct, clst, k1, k0, k1t, k0t;
  T3 alpha[2][4], beta[2][4];
  double ct, st, xp_fac, ix_fac, x_fac, S0inv, weff[2];
  int32_t n_eff, pad;
};

// Pattern maps of one interferometer (as pattern_map) and their derivatives
// along its bisector angle.
__host__ __device__ inline void pattern_map_t(double gamma, double zeta, double c2p, double s2p,
                                              T3 al[4], T3 be[4]) {
  const double sz = sin(zeta), s2g = sin(2.0 * gamma), c2g = cos(2.0 * gamma);
  const double v_al[4] = {sz * s2g * c2p, -sz * c2g * c2p, sz * s2g * s2p, -sz * c2g * s2p};
  const double v_be[4] = {-sz * s2g * s2p, sz * c2g * s2p, sz * s2g * c2p, -sz * c2g * c2p};
  // d/dgamma: s2g -> 2 c2g, c2g -> -2 s2g
  const double g_al[4] = {2.0 * sz * c2g * c2p, 2.0 * sz * s2g * c2p, 2.0 * sz * c2g * s2p,
                          2.0 * sz * s2g * s2p};
  const double g_be[4] = {-2.0 * sz * c2g * s2p, -2.0 * sz * s2g * s2p, 2.0 * sz * c2g * c2p,
                          2.0 * sz * s2g * c2p};
  for (int i = 0; i < 4; ++i) {
    al[i] = T3{v_al[i], {0.0, 0.0, g_al[i]}};
    be[i] = T3{v_be[i], {0.0, 0.0, g_be[i]}};
  }
}

__host__ __device__ inline void site_setup_adj(const double* p, const SiteDesc& sd, const EventC& ec,
                                               SiteA& sa) {
  const double th = p[3], ph = p[4], psi = p[6];
  const double c2p = cos(2.0 * psi), s2p = sin(2.0 * psi);
  const double cdl = cos(sd.lon - ph), sdl = sin(sd.lon - ph);
  sa.cdl = T3{cdl, {0.0, -sdl, 0.0}};
  sa.sdl = T3{sdl, {0.0, cdl, 0.0}};
  const double ct = cos(th), st = sin(th), sl = sin(sd.lat), cl = cos(sd.lat);
  sa.ct = ct; sa.st = st;
  const T3 tsl = T3{sl, {cl, 0.0, 0.0}}, tcl = T3{cl, {-sl, 0.0, 0.0}};
  sa.sl = tsl;
  sa.cl = tcl;
  sa.slct = ct * tsl;
  sa.clst = st * tcl;
  sa.k1 = (-kREarthS * st) * tcl;
  sa.k0 = (-kREarthS * ct) * tsl;
  sa.k1t = (-kREarthS * ct) * tcl;
  sa.k0t = (kREarthS * st) * tsl;
  sa.xp_fac = exp(4.14 * (log(ec.piM) + log(sd.f0)));
  sa.ix_fac = sd.f0 * ec.piM;
  sa.x_fac = 1.0 / sa.ix_fac;
  sa.S0inv = 1.0 / sd.S0;
  if (sd.shape == 1) {
    T3 al[3][4], be[3][4];
    for (int k = 0; k < 3; ++k)
      pattern_map_t(sd.gamma + kPi / 6.0 + kTwoPi * k / 3.0, kPi / 3.0, c2p, s2p, al[k], be[k]);
    for (int j = 0; j < 4; ++j) {
      sa.alpha[0][j] = al[0][j] + al[1][j]; sa.beta[0][j] = be[0][j] + be[1][j];
      sa.alpha[1][j] = al[0][j] - al[1][j]; sa.beta[1][j] = be[0][j] - be[1][j];
    }
    sa.weff[0] = 1.5; sa.weff[1] = 0.5;
    sa.n_eff = 2;
  } else {
    pattern_map_t(sd.gamma, sd.zeta, c2p, s2p, sa.alpha[0], sa.beta[0]);
    for (int j = 0; j < 4; ++j) { sa.alpha[1][j] = t3c(0.0); sa.beta[1][j] = t3c(0.0); }
    sa.weff[0] = 1.0; sa.weff[1] = 0.0;
    sa.n_eff = 1;
  }
  sa.pad = 0;
}

// Accumulator slots of one site: sum Gbar dGamma along (lat, lon, gamma,
// ln S0), dSNR^2 along the same four, and SNR^2 itself.
enum { kAdjT = 0, kAdjS = 4, kAdjW = 8, kAdjN = 9 };

// ------------------------------------------------------ one grid point
// Adds the contribution of grid point k and site sa to acc[kAdjN].  Gb is the
// symmetric P x P matrix Gbar of the event (row-major).
//
// The derivative vectors D_b (b < 8) are built from the pattern values
// F = (Fp, Fx) and their hour-angle and theta derivatives FH, Ft, and from
// the arrival-time derivatives dH, dT; the phase-only ones are i Q c_i.  With
// z = Gbar D held fixed, sum_b Re(dD_b . z_b^*) is linear in the derivatives
// of those building blocks, so the point first forms the weights kappa of
// the building blocks (reverse mode through the D formulas, values only) and
// then contracts them with the building blocks' tangents along latitude,
// longitude and gamma (forward mode through the site geometry).
// Per grid point, shared by all sites: the point quantities, and
//   gc_a = sum_i Gbar_{a, 8+i} c_i  (a < 8),   cgc = sum_ij c_i Gbar_{8+i, 8+j} c_j,
// so that with D_{8+i} = i Q c_i the rows z_a = (Gbar D)_a for a < 8 and the
// contraction c . z_{8:} of the phase-only rows need only Gbar[:8, :8], gc
// and cgc (Gbar symmetric).
struct AdjPoint {
  Point q;
  double gc[8], cgc;
};

template <bool TIDAL, bool ROT>
__host__ __device__ inline void adjoint_point_setup(const EventC& ec, const double* Gb, int32_t k,
                                                    AdjPoint& ap) {
  constexpr int NPI = TIDAL ? 5 : 3;
  constexpr int P = 8 + NPI;
  point_setup(ec, k, true, ROT, ap.q);
  double c[NPI];
  phase_only_coefficients<TIDAL>(ec, ap.q, c);
  double cg[NPI];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NPI; ++i) t = fma(Gb[a * P + 8 + i], c[i], t);
    ap.gc[a] = t;
  }
#pragma unroll
  for (int i = 0; i < NPI; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < NPI; ++j) t = fma(Gb[(8 + i) * P + 8 + j], c[j], t);
    cg[i] = t;
  }
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NPI; ++i) t = fma(c[i], cg[i], t);
  ap.cgc = t;
}

// Adds the contribution of one site at the point to acc[kAdjN].
template <bool TIDAL>
__host__ __device__ inline void adjoint_site(const EventC& ec, const SiteA& sa, const double* Gb,
                                             const AdjPoint& ap, double* acc) {
  constexpr int NPI = TIDAL ? 5 : 3;
  constexpr int P = 8 + NPI;
  const Point& q = ap.q;
  // hour angle, pattern vectors, arrival-time offset derivatives (tangents)
  const T3 cH = q.cth * sa.cdl - q.sth * sa.sdl;
  const T3 sH = q.sth * sa.cdl + q.cth * sa.sdl;
  const T3 EX = cH, EY = -(sa.ct * sH), NX = -(sa.sl * sH), NY = -(sa.slct * cH + sa.clst);
  T3 Pv[4], PH[4], Pt[4];
  Pv[0] = 0.5 * (EX * EX - NX * NX - EY * EY + NY * NY);
  Pv[1] = EX * NX - EY * NY;
  Pv[2] = EX * EY - NX * NY;
  Pv[3] = EX * NY + NX * EY;
  {
    const T3 EXh = -sH, EYh = -(sa.ct * cH), NXh = -(sa.sl * cH), NYh = sa.slct * sH;
    PH[0] = EX * EXh - NX * NXh - EY * EYh + NY * NYh;
    PH[1] = EXh * NX + EX * NXh - EYh * NY - EY * NYh;
    PH[2] = EXh * EY + EX * EYh - NXh * NY - NX * NYh;
    PH[3] = EXh * NY + EX * NYh + NXh * EY + NX * EYh;
    // d/dtheta of EY and NY (theta is the source angle, not a detector parameter)
    const T3 EYt = sa.st * sH, NYt = sa.st * (sa.sl * cH) - sa.ct * sa.cl;
    Pt[0] = -(EY * EYt) + NY * NYt;
    Pt[1] = -(EYt * NY + EY * NYt);
    Pt[2] = EX * EYt - NX * NYt;
    Pt[3] = EX * NYt + NX * EYt;
  }
  const T3 dH = -(sa.k1 * sH);
  const T3 dT = fmat(sa.k1t, cH, sa.k0t);
  const double om0 = psd_weight_of(sa.xp_fac, 0.0, sa.ix_fac, sa.x_fac, sa.S0inv, q);
  const double tf = q.tf;
  const double phMc = fma(tf * dH.v, q.gMc, q.pMc), phEta = fma(tf * dH.v, q.gEta, q.pEta);
  const double phT = tf * dT.v, phP = -tf * dH.v, phTc = tf * fma(kOmegaE, dH.v, 1.0);
  const double cplus = ec.cplus, ccross = ec.ccross, dcp = ec.dcplus, dcx = ec.dcross;
  const double dlnA = ec.dlnA_dMc, idL = ec.inv_dL;
  for (int j = 0; j < sa.n_eff; ++j) {
    // compiler barrier: the constants below are loaded when needed rather
    // than all at once (register pressure)
    asm volatile("" ::: "memory");
    const double om = om0 * sa.weff[j];
    const T3 Fp = dot4t(sa.alpha[j], Pv), Fx = dot4t(sa.beta[j], Pv);
    const T3 FpH = dot4t(sa.alpha[j], PH), FxH = dot4t(sa.beta[j], PH);
    const T3 Fpt = dot4t(sa.alpha[j], Pt), Fxt = dot4t(sa.beta[j], Pt);
    const double Qr = cplus * Fp.v, Qi = ccross * Fx.v;
    const double QHr = cplus * FpH.v, QHi = ccross * FxH.v;
    const double Qtr = cplus * Fpt.v, Qti = ccross * Fxt.v;
    // D values (as in accumulate_point)
    double Dr[8], Di[8];
    Dr[0] = fma(Qr, dlnA, fma(QHr, q.gMc, -Qi * phMc));
    Di[0] = fma(Qi, dlnA, fma(QHi, q.gMc, Qr * phMc));
    Dr[1] = fma(QHr, q.gEta, -Qi * phEta);
    Di[1] = fma(QHi, q.gEta, Qr * phEta);
    Dr[2] = -Qr * idL;
    Di[2] = -Qi * idL;
    Dr[3] = fma(-Qi, phT, Qtr);
    Di[3] = fma(Qr, phT, Qti);
    Dr[4] = fma(-Qi, phP, -QHr);
    Di[4] = fma(Qr, phP, -QHi);
    Dr[5] = dcp * Fp.v;
    Di[5] = dcx * Fx.v;
    Dr[6] = 2.0 * cplus * Fx.v;
    Di[6] = -2.0 * ccross * Fp.v;
    Dr[7] = fma(kOmegaE, QHr, -Qi * phTc);
    Di[7] = fma(kOmegaE, QHi, Qr * phTc);
    // z = Gbar D for rows a < 8, and c . z over the phase-only rows, from
    // Gbar[:8, :8], gc and cgc (see AdjPoint)
    double zr[8], zi[8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      asm volatile("" ::: "memory");
      double sr = -Qi * ap.gc[a], si = Qr * ap.gc[a];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        sr = fma(Gb[a * P + b], Dr[b], sr);
        si = fma(Gb[a * P + b], Di[b], si);
      }
      zr[a] = sr;
      zi[a] = si;
    }
    double czr = -Qi * ap.cgc, czi = Qr * ap.cgc;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      czr = fma(ap.gc[b], Dr[b], czr);
      czi = fma(ap.gc[b], Di[b], czi);
    }
    // Re(D^H z) for the ln S0 term
    double dz = fma(-Qi, czr, Qr * czi);
#pragma unroll
    for (int b = 0; b < 8; ++b) dz = fma(Dr[b], zr[b], fma(Di[b], zi[b], dz));
    // weights of the building blocks in sum_b Re(D_b z_b^*) (+ the phase-only rows)
    const double kQr = fma(dlnA, zr[0], fma(phMc, zi[0], fma(phEta, zi[1], fma(-idL, zr[2],
                       fma(phT, zi[3], fma(phP, zi[4], fma(phTc, zi[7], czi)))))));
    const double kQi = fma(-phMc, zr[0], fma(dlnA, zi[0], fma(-phEta, zr[1], fma(-idL, zi[2],
                       fma(-phT, zr[3], fma(-phP, zr[4], fma(-phTc, zr[7], -czr)))))));
    const double kQHr = fma(q.gMc, zr[0], fma(q.gEta, zr[1], fma(kOmegaE, zr[7], -zr[4])));
    const double kQHi = fma(q.gMc, zi[0], fma(q.gEta, zi[1], fma(kOmegaE, zi[7], -zi[4])));
    const double kQtr = zr[3], kQti = zi[3];
    const double kphMc = fma(-Qi, zr[0], Qr * zi[0]);
    const double kphEta = fma(-Qi, zr[1], Qr * zi[1]);
    const double kphT = fma(-Qi, zr[3], Qr * zi[3]);
    const double kphP = fma(-Qi, zr[4], Qr * zi[4]);
    const double kphTc = fma(-Qi, zr[7], Qr * zi[7]);
    // ... mapped to the pattern values and the arrival-time derivatives
    const double kFp = fma(cplus, kQr, fma(dcp, zr[5], -2.0 * ccross * zi[6]));
    const double kFx = fma(ccross, kQi, fma(dcx, zi[5], 2.0 * cplus * zr[6]));
    const double kFpH = cplus * kQHr, kFxH = ccross * kQHi;
    const double kFpt = cplus * kQtr, kFxt = ccross * kQti;
    const double kdH = tf * fma(q.gMc, kphMc, fma(q.gEta, kphEta, fma(kOmegaE, kphTc, -kphP)));
    const double kdT = tf * kphT;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      double t = kFp * Fp.d[x];
      t = fma(kFx, Fx.d[x], t);
      t = fma(kFpH, FpH.d[x], t);
      t = fma(kFxH, FxH.d[x], t);
      t = fma(kFpt, Fpt.d[x], t);
      t = fma(kFxt, Fxt.d[x], t);
      t = fma(kdH, dH.d[x], t);
      t = fma(kdT, dT.d[x], t);
      acc[kAdjT + x] = fma(2.0 * om, t, acc[kAdjT + x]);
      acc[kAdjS + x] = fma(2.0 * om, fma(Qr * cplus, Fp.d[x], Qi * ccross * Fx.d[x]), acc[kAdjS + x]);
    }
    const double q2 = fma(Qr, Qr, Qi * Qi);
    acc[kAdjT + 3] = fma(-om, dz, acc[kAdjT + 3]);
    acc[kAdjS + 3] = fma(-om, q2, acc[kAdjS + 3]);
    acc[kAdjW] = fma(om, q2, acc[kAdjW]);
  }
}

// One grid point and one site (host checks).
template <bool TIDAL, bool ROT>
__host__ __device__ inline void adjoint_point(const EventC& ec, const SiteA& sa, const double* Gb,
                                              int32_t k, double* acc) {
  AdjPoint ap;
  adjoint_point_setup<TIDAL, ROT>(ec, Gb, k, ap);
  adjoint_site<TIDAL>(ec, sa, Gb, ap, acc);
}

}  // namespace gwf

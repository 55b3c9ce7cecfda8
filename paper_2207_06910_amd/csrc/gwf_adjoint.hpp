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
  int32_t n_eff, tab_kind;
  const double* tab_f;      // sampled noise curve (tab_kind 1 PSD, 2 ASD), as SiteC
  const double* tab_S;
  int64_t tab_n;
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

// arm_on as for site_setup.
__host__ __device__ inline void site_setup_adj(const double* p, const SiteDesc& sd, const EventC& ec,
                                               SiteA& sa, uint32_t arm_on = 7u) {
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
  sa.tab_kind = sd.psd_kind;
  sa.tab_f = sd.tab_f;
  sa.tab_S = sd.tab_S;
  sa.tab_n = sd.tab_n;
  if (sd.shape == 1) {
    T3 al[3][4], be[3][4];
    for (int k = 0; k < 3; ++k)
      pattern_map_t(sd.gamma + kPi / 6.0 + kTwoPi * k / 3.0, kPi / 3.0, c2p, s2p, al[k], be[k]);
    if ((arm_on & 7u) == 7u) {
      for (int j = 0; j < 4; ++j) {
        sa.alpha[0][j] = al[0][j] + al[1][j]; sa.beta[0][j] = be[0][j] + be[1][j];
        sa.alpha[1][j] = al[0][j] - al[1][j]; sa.beta[1][j] = be[0][j] - be[1][j];
      }
      sa.weff[0] = 1.5; sa.weff[1] = 0.5;
      sa.n_eff = 2;
    } else {
      int m = 0;
      for (int k = 0; k < 3; ++k)
        if (arm_on >> k & 1u) {
          for (int j = 0; j < 4; ++j) { sa.alpha[m][j] = al[k][j]; sa.beta[m][j] = be[k][j]; }
          sa.weff[m] = 1.0;
          ++m;
        }
      for (int r = m; r < 2; ++r) {
        for (int j = 0; j < 4; ++j) { sa.alpha[r][j] = t3c(0.0); sa.beta[r][j] = t3c(0.0); }
        sa.weff[r] = 0.0;
      }
      sa.n_eff = m;
    }
  } else {
    pattern_map_t(sd.gamma, sd.zeta, c2p, s2p, sa.alpha[0], sa.beta[0]);
    for (int j = 0; j < 4; ++j) { sa.alpha[1][j] = t3c(0.0); sa.beta[1][j] = t3c(0.0); }
    sa.weff[0] = 1.0; sa.weff[1] = 0.0;
    sa.n_eff = (arm_on & 1u) ? 1 : 0;
  }
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

template <int NPI, bool ROT>
__host__ __device__ inline void adjoint_point_setup(const EventC& ec, const double* Gb, int32_t k,
                                                    AdjPoint& ap) {
  constexpr int P = 8 + NPI;
  point_setup<true, false, PhaseOnly<NPI>::ecc>(ec, k, true, ROT, ap.q);
  double c[NPI];
  phase_only_coefficients<NPI>(ec, ap.q, c);
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
//
// Order of the work: the site geometry is evaluated as values only; for each
// effective interferometer the derivative vectors, z and the reverse weights
// kappa of the building blocks are formed and folded (times 2w) into the
// adjoints of the site's pattern vectors P, PH, Pt (4 each) and of dH, dT,
// since Fp = alpha . P etc. are linear in them; gamma moves only alpha and
// beta, so its terms are taken per interferometer from their gamma
// derivatives.  After the last interferometer, one forward pass through the
// geometry gives the latitude and longitude tangents of P, PH, Pt, dH and dT,
// contracted with those adjoints.  Only the values and the adjoints are live
// across the interferometers.
template <int NPI>
__host__ __device__ inline void adjoint_site(const EventC& ec, const SiteA& sa, const double* Gb,
                                             const AdjPoint& ap, double* acc) {
  constexpr int P = 8 + NPI;
  const Point& q = ap.q;
  // hour angle, pattern vectors and arrival-time derivatives: values
  double Pv[4], PH[4], Pt[4], dHv, dTv;
  {
    const double cH = q.cth * sa.cdl.v - q.sth * sa.sdl.v;
    const double sH = q.sth * sa.cdl.v + q.cth * sa.sdl.v;
    const double EX = cH, EY = -(sa.ct * sH), NX = -(sa.sl.v * sH), NY = -(sa.slct.v * cH + sa.clst.v);
    Pv[0] = 0.5 * (EX * EX - NX * NX - EY * EY + NY * NY);
    Pv[1] = EX * NX - EY * NY;
    Pv[2] = EX * EY - NX * NY;
    Pv[3] = EX * NY + NX * EY;
    const double EXh = -sH, EYh = -(sa.ct * cH), NXh = -(sa.sl.v * cH), NYh = sa.slct.v * sH;
    PH[0] = EX * EXh - NX * NXh - EY * EYh + NY * NYh;
    PH[1] = EXh * NX + EX * NXh - EYh * NY - EY * NYh;
    PH[2] = EXh * EY + EX * EYh - NXh * NY - NX * NYh;
    PH[3] = EXh * NY + EX * NYh + NXh * EY + NX * EYh;
    const double EYt = sa.st * sH, NYt = sa.st * (sa.sl.v * cH) - sa.ct * sa.cl.v;
    Pt[0] = -(EY * EYt) + NY * NYt;
    Pt[1] = -(EYt * NY + EY * NYt);
    Pt[2] = EX * EYt - NX * NYt;
    Pt[3] = EX * NYt + NX * EYt;
    dHv = -(sa.k1.v * sH);
    dTv = fma(sa.k1t.v, cH, sa.k0t.v);
  }
  const double om0 = sa.tab_kind ? table_weight(sa.tab_f, sa.tab_S, sa.tab_n, sa.tab_kind, sa.S0inv, q.w4A2, q.f)
                                 : psd_weight_of(sa.xp_fac, 0.0, sa.ix_fac, sa.x_fac, sa.S0inv, q);
  const double tf = q.tf;
  const double phMc = fma(tf * dHv, q.gMc, q.pMc), phEta = fma(tf * dHv, q.gEta, q.pEta);
  const double phT = tf * dTv, phP = -tf * dHv, phTc = tf * fma(kOmegaE, dHv, 1.0);
  const double cplus = ec.cplus, ccross = ec.ccross, dcp = ec.dcplus, dcx = ec.dcross;
  const double dlnA = ec.dlnA_dMc, idL = ec.inv_dL;
  // adjoints, summed over the interferometers: Gbar:dGamma (b) and SNR^2 (s)
  double bP[4] = {0.0, 0.0, 0.0, 0.0}, bPH[4] = {0.0, 0.0, 0.0, 0.0}, bPt[4] = {0.0, 0.0, 0.0, 0.0};
  double sP[4] = {0.0, 0.0, 0.0, 0.0};
  double bdH = 0.0, bdT = 0.0, bgam = 0.0, sgam = 0.0;
  // at most two effective interferometers; unrolled, with the count the same
  // for every lane (the second pass is skipped as a whole where unused)
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= sa.n_eff) break;
    // compiler barrier: the constants below are loaded when needed rather
    // than all at once (register pressure)
    asm volatile("" ::: "memory");
    const double om = om0 * sa.weff[j];
    double al[4], be[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      al[i] = sa.alpha[j][i].v;
      be[i] = sa.beta[j][i].v;
    }
    const double Fp = dot4(al, Pv), Fx = dot4(be, Pv);
    const double FpH = dot4(al, PH), FxH = dot4(be, PH);
    const double Fpt = dot4(al, Pt), Fxt = dot4(be, Pt);
    const double Qr = cplus * Fp, Qi = ccross * Fx;
    const double QHr = cplus * FpH, QHi = ccross * FxH;
    const double Qtr = cplus * Fpt, Qti = ccross * Fxt;
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
    Dr[5] = dcp * Fp;
    Di[5] = dcx * Fx;
    Dr[6] = 2.0 * cplus * Fx;
    Di[6] = -2.0 * ccross * Fp;
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
    const double f = 2.0 * om;
    const double kFp = f * fma(cplus, kQr, fma(dcp, zr[5], -2.0 * ccross * zi[6]));
    const double kFx = f * fma(ccross, kQi, fma(dcx, zi[5], 2.0 * cplus * zr[6]));
    const double kFpH = f * (cplus * kQHr), kFxH = f * (ccross * kQHi);
    const double kFpt = f * (cplus * kQtr), kFxt = f * (ccross * kQti);
    bdH = fma(f * tf, fma(q.gMc, kphMc, fma(q.gEta, kphEta, fma(kOmegaE, kphTc, -kphP))), bdH);
    bdT = fma(f * tf, kphT, bdT);
    const double sFp = f * (Qr * cplus), sFx = f * (Qi * ccross);
    double ag[4], bg[4];                      // d alpha / d gamma, d beta / d gamma
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bP[i] = fma(kFp, al[i], fma(kFx, be[i], bP[i]));
      bPH[i] = fma(kFpH, al[i], fma(kFxH, be[i], bPH[i]));
      bPt[i] = fma(kFpt, al[i], fma(kFxt, be[i], bPt[i]));
      sP[i] = fma(sFp, al[i], fma(sFx, be[i], sP[i]));
      ag[i] = sa.alpha[j][i].d[2];
      bg[i] = sa.beta[j][i].d[2];
    }
    const double gFp = dot4(ag, Pv), gFx = dot4(bg, Pv);
    bgam = fma(kFp, gFp, fma(kFx, gFx, fma(kFpH, dot4(ag, PH), fma(kFxH, dot4(bg, PH),
           fma(kFpt, dot4(ag, Pt), fma(kFxt, dot4(bg, Pt), bgam))))));
    sgam = fma(sFp, gFp, fma(sFx, gFx, sgam));
    const double q2 = fma(Qr, Qr, Qi * Qi);
    acc[kAdjT + 3] = fma(-om, dz, acc[kAdjT + 3]);
    acc[kAdjS + 3] = fma(-om, q2, acc[kAdjS + 3]);
    acc[kAdjW] = fma(om, q2, acc[kAdjW]);
  }
  // latitude and longitude tangents of the geometry, contracted with the adjoints
  asm volatile("" ::: "memory");
  const T3 cH = q.cth * sa.cdl - q.sth * sa.sdl;
  const T3 sH = q.sth * sa.cdl + q.cth * sa.sdl;
  const T3 EX = cH, EY = -(sa.ct * sH), NX = -(sa.sl * sH), NY = -(sa.slct * cH + sa.clst);
  double tb[2] = {0.0, 0.0}, ts[2] = {0.0, 0.0};
  {
    const T3 P0 = 0.5 * (EX * EX - NX * NX - EY * EY + NY * NY);
    const T3 P1 = EX * NX - EY * NY;
    const T3 P2 = EX * EY - NX * NY;
    const T3 P3 = EX * NY + NX * EY;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      tb[x] = fma(bP[0], P0.d[x], fma(bP[1], P1.d[x], fma(bP[2], P2.d[x], bP[3] * P3.d[x])));
      ts[x] = fma(sP[0], P0.d[x], fma(sP[1], P1.d[x], fma(sP[2], P2.d[x], sP[3] * P3.d[x])));
    }
  }
  {
    const T3 EXh = -sH, EYh = -(sa.ct * cH), NXh = -(sa.sl * cH), NYh = sa.slct * sH;
    const T3 H0 = EX * EXh - NX * NXh - EY * EYh + NY * NYh;
    const T3 H1 = EXh * NX + EX * NXh - EYh * NY - EY * NYh;
    const T3 H2 = EXh * EY + EX * EYh - NXh * NY - NX * NYh;
    const T3 H3 = EXh * NY + EX * NYh + NXh * EY + NX * EYh;
#pragma unroll
    for (int x = 0; x < 2; ++x)
      tb[x] = fma(bPH[0], H0.d[x], fma(bPH[1], H1.d[x], fma(bPH[2], H2.d[x], fma(bPH[3], H3.d[x], tb[x]))));
  }
  {
    const T3 EYt = sa.st * sH, NYt = sa.st * (sa.sl * cH) - sa.ct * sa.cl;
    const T3 T0 = -(EY * EYt) + NY * NYt;
    const T3 T1 = -(EYt * NY + EY * NYt);
    const T3 T2 = EX * EYt - NX * NYt;
    const T3 T3v = EX * NYt + NX * EYt;
#pragma unroll
    for (int x = 0; x < 2; ++x)
      tb[x] = fma(bPt[0], T0.d[x], fma(bPt[1], T1.d[x], fma(bPt[2], T2.d[x], fma(bPt[3], T3v.d[x], tb[x]))));
  }
  const T3 dH = -(sa.k1 * sH);
  const T3 dT = fmat(sa.k1t, cH, sa.k0t);
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    acc[kAdjT + x] += fma(bdH, dH.d[x], fma(bdT, dT.d[x], tb[x]));
    acc[kAdjS + x] += ts[x];
  }
  acc[kAdjT + 2] += bgam;
  acc[kAdjS + 2] += sgam;
}

// One grid point and one site (host checks).
template <int NPI, bool ROT>
__host__ __device__ inline void adjoint_point(const EventC& ec, const SiteA& sa, const double* Gb,
                                              int32_t k, double* acc) {
  AdjPoint ap;
  adjoint_point_setup<NPI, ROT>(ec, Gb, k, ap);
  adjoint_site<NPI>(ec, sa, Gb, ap, acc);
}

}  // namespace gwf

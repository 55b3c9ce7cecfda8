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
// Jacobian is stored.  Reverse mode all the way: the weights of the building
// blocks (the pattern vectors P, their hour-angle and theta derivatives PH,
// Pt, and the arrival-time derivatives dH, dT) are taken back to the site's
// local frame vectors (the E/N components of the polarisation frame and
// their H and theta derivatives), whose derivatives along latitude and
// longitude are a handful of closed forms (the longitude enters only through
// the hour angle, so d/dlon = d/dH); gamma moves only the pattern maps.
// Along ln S0 only the weight changes, dw = -w, which gives
// -sum w Re(D^H z) in closed form.
#pragma once

#include "gwf_model.hpp"

namespace gwf {

// ----------------------------------------------------- site constants
// The per-(event, site) constants of site_setup that the adjoint needs, and
// the derivatives of the pattern maps along gamma.
struct SiteA {
  double cdl, sdl;                       // cos, sin of (site longitude - phi)
  double ct, st, sl, cl, slct, clst;     // cos th, sin th, sin lat, cos lat, sin lat cos th, cos lat sin th
  double k1, k1t, k0t;                   // Delta = k1 cos H + k0, dDelta/dth = k1t cos H + k0t
  double alpha[2][4], beta[2][4];        // pattern maps of the effective interferometers
  double alpha_g[2][4], beta_g[2][4];    // and their derivatives along gamma
  double xp_fac, ix_fac, x_fac, S0inv, weff[2];
  int32_t n_eff, tab_kind;
  const double* tab_f;                   // sampled noise curve (tab_kind 1 PSD, 2 ASD), as SiteC
  const double* tab_S;
  int64_t tab_n;
};

// Pattern maps of one interferometer (as pattern_map) and their derivatives
// along its bisector angle gamma.
__host__ __device__ inline void pattern_map_g(double gamma, double zeta, double c2p, double s2p, double al[4],
                                              double be[4], double alg[4], double beg[4]) {
  pattern_map(gamma, zeta, c2p, s2p, al, be);
  const double sz = sin(zeta), s2g = sin(2.0 * gamma), c2g = cos(2.0 * gamma);
  // d/dgamma: s2g -> 2 c2g, c2g -> -2 s2g
  alg[0] = 2.0 * sz * c2g * c2p; alg[1] = 2.0 * sz * s2g * c2p; alg[2] = 2.0 * sz * c2g * s2p;
  alg[3] = 2.0 * sz * s2g * s2p;
  beg[0] = -2.0 * sz * c2g * s2p; beg[1] = -2.0 * sz * s2g * s2p; beg[2] = 2.0 * sz * c2g * c2p;
  beg[3] = 2.0 * sz * s2g * c2p;
}

// arm_on as for site_setup.
__host__ __device__ inline void site_setup_adj(const double* p, const SiteDesc& sd, const EventC& ec,
                                               SiteA& sa, uint32_t arm_on = 7u) {
  const double th = p[3], ph = p[4], psi = p[6];
  const double c2p = cos(2.0 * psi), s2p = sin(2.0 * psi);
  sa.cdl = cos(sd.lon - ph);
  sa.sdl = sin(sd.lon - ph);
  const double ct = cos(th), st = sin(th), sl = sin(sd.lat), cl = cos(sd.lat);
  sa.ct = ct; sa.st = st; sa.sl = sl; sa.cl = cl;
  sa.slct = sl * ct;
  sa.clst = cl * st;
  sa.k1 = -kREarthS * cl * st;
  sa.k1t = -kREarthS * cl * ct;
  sa.k0t = kREarthS * sl * st;
  sa.xp_fac = exp(4.14 * (log(ec.piM) + log(sd.f0)));
  sa.ix_fac = sd.f0 * ec.piM;
  sa.x_fac = 1.0 / sa.ix_fac;
  sa.S0inv = 1.0 / sd.S0;
  sa.tab_kind = sd.psd_kind;
  sa.tab_f = sd.tab_f;
  sa.tab_S = sd.tab_S;
  sa.tab_n = sd.tab_n;
  for (int r = 0; r < 2; ++r)
    for (int j = 0; j < 4; ++j) sa.alpha[r][j] = sa.beta[r][j] = sa.alpha_g[r][j] = sa.beta_g[r][j] = 0.0;
  if (sd.shape == 1) {
    double al[3][4], be[3][4], alg[3][4], beg[3][4];
    for (int k = 0; k < 3; ++k)
      pattern_map_g(sd.gamma + kPi / 6.0 + kTwoPi * k / 3.0, kPi / 3.0, c2p, s2p, al[k], be[k], alg[k], beg[k]);
    if ((arm_on & 7u) == 7u) {
      for (int j = 0; j < 4; ++j) {
        sa.alpha[0][j] = al[0][j] + al[1][j]; sa.beta[0][j] = be[0][j] + be[1][j];
        sa.alpha[1][j] = al[0][j] - al[1][j]; sa.beta[1][j] = be[0][j] - be[1][j];
        sa.alpha_g[0][j] = alg[0][j] + alg[1][j]; sa.beta_g[0][j] = beg[0][j] + beg[1][j];
        sa.alpha_g[1][j] = alg[0][j] - alg[1][j]; sa.beta_g[1][j] = beg[0][j] - beg[1][j];
      }
      sa.weff[0] = 1.5; sa.weff[1] = 0.5;
      sa.n_eff = 2;
    } else {
      int m = 0;
      for (int k = 0; k < 3; ++k)
        if (arm_on >> k & 1u) {
          for (int j = 0; j < 4; ++j) {
            sa.alpha[m][j] = al[k][j]; sa.beta[m][j] = be[k][j];
            sa.alpha_g[m][j] = alg[k][j]; sa.beta_g[m][j] = beg[k][j];
          }
          sa.weff[m] = 1.0;
          ++m;
        }
      for (int r = m; r < 2; ++r) sa.weff[r] = 0.0;
      sa.n_eff = m;
    }
  } else {
    pattern_map_g(sd.gamma, sd.zeta, c2p, s2p, sa.alpha[0], sa.beta[0], sa.alpha_g[0], sa.beta_g[0]);
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
    // the site's E/N frame components of the polarisation frame and their H
    // and theta derivatives (formed again for the reverse pass below rather
    // than kept live across the interferometers)
    const double cH = q.cth * sa.cdl - q.sth * sa.sdl;
    const double sH = q.sth * sa.cdl + q.cth * sa.sdl;
    const double EX = cH, EY = -(sa.ct * sH), NX = -(sa.sl * sH), NY = -(sa.slct * cH + sa.clst);
    const double EXh = -sH, EYh = -(sa.ct * cH), NXh = -(sa.sl * cH), NYh = sa.slct * sH;
    const double EYt = sa.st * sH, NYt = sa.st * (sa.sl * cH) - sa.ct * sa.cl;
    Pv[0] = 0.5 * (EX * EX - NX * NX - EY * EY + NY * NY);
    Pv[1] = EX * NX - EY * NY;
    Pv[2] = EX * EY - NX * NY;
    Pv[3] = EX * NY + NX * EY;
    PH[0] = EX * EXh - NX * NXh - EY * EYh + NY * NYh;
    PH[1] = EXh * NX + EX * NXh - EYh * NY - EY * NYh;
    PH[2] = EXh * EY + EX * EYh - NXh * NY - NX * NYh;
    PH[3] = EXh * NY + EX * NYh + NXh * EY + NX * EYh;
    Pt[0] = -(EY * EYt) + NY * NYt;
    Pt[1] = -(EYt * NY + EY * NYt);
    Pt[2] = EX * EYt - NX * NYt;
    Pt[3] = EX * NYt + NX * EYt;
    dHv = -(sa.k1 * sH);
    dTv = fma(sa.k1t, cH, sa.k0t);
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
      al[i] = sa.alpha[j][i];
      be[i] = sa.beta[j][i];
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
      ag[i] = sa.alpha_g[j][i];
      bg[i] = sa.beta_g[j][i];
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
  // reverse pass through the geometry: the weights of the pattern vectors
  // (bP, bPH, bPt; sP for SNR^2) taken back to the frame components EX, EY,
  // NX, NY, their H derivatives (h) and theta derivatives (t) ...
  asm volatile("" ::: "memory");
  const double cH = q.cth * sa.cdl - q.sth * sa.sdl;
  const double sH = q.sth * sa.cdl + q.cth * sa.sdl;
  const double EX = cH, EY = -(sa.ct * sH), NX = -(sa.sl * sH), NY = -(sa.slct * cH + sa.clst);
  const double EXh = -sH, EYh = -(sa.ct * cH), NXh = -(sa.sl * cH), NYh = sa.slct * sH;
  const double EYt = sa.st * sH, NYt = sa.st * (sa.sl * cH) - sa.ct * sa.cl;
  const double aEX = fma(bP[0], EX, fma(bP[1], NX, fma(bP[2], EY, fma(bP[3], NY, fma(bPH[0], EXh,
                     fma(bPH[1], NXh, fma(bPH[2], EYh, fma(bPH[3], NYh, fma(bPt[2], EYt, bPt[3] * NYt)))))))));
  const double aEY = fma(-bP[0], EY, fma(-bP[1], NY, fma(bP[2], EX, fma(bP[3], NX, fma(-bPH[0], EYh,
                     fma(-bPH[1], NYh, fma(bPH[2], EXh, fma(bPH[3], NXh, fma(-bPt[0], EYt, -bPt[1] * NYt)))))))));
  const double aNX = fma(-bP[0], NX, fma(bP[1], EX, fma(-bP[2], NY, fma(bP[3], EY, fma(-bPH[0], NXh,
                     fma(bPH[1], EXh, fma(-bPH[2], NYh, fma(bPH[3], EYh, fma(-bPt[2], NYt, bPt[3] * EYt)))))))));
  const double aNY = fma(bP[0], NY, fma(-bP[1], EY, fma(-bP[2], NX, fma(bP[3], EX, fma(bPH[0], NYh,
                     fma(-bPH[1], EYh, fma(-bPH[2], NXh, fma(bPH[3], EXh, fma(bPt[0], NYt, -bPt[1] * EYt)))))))));
  const double aEXh = fma(bPH[0], EX, fma(bPH[1], NX, fma(bPH[2], EY, bPH[3] * NY)));
  const double aEYh = fma(-bPH[0], EY, fma(-bPH[1], NY, fma(bPH[2], EX, bPH[3] * NX)));
  const double aNXh = fma(-bPH[0], NX, fma(bPH[1], EX, fma(-bPH[2], NY, bPH[3] * EY)));
  const double aNYh = fma(bPH[0], NY, fma(-bPH[1], EY, fma(-bPH[2], NX, bPH[3] * EX)));
  const double aEYt = fma(-bPt[0], EY, fma(-bPt[1], NY, fma(bPt[2], EX, bPt[3] * NX)));
  const double aNYt = fma(bPt[0], NY, fma(-bPt[1], EY, fma(-bPt[2], NX, bPt[3] * EX)));
  const double sEX = fma(sP[0], EX, fma(sP[1], NX, fma(sP[2], EY, sP[3] * NY)));
  const double sEY = fma(-sP[0], EY, fma(-sP[1], NY, fma(sP[2], EX, sP[3] * NX)));
  const double sNX = fma(-sP[0], NX, fma(sP[1], EX, fma(-sP[2], NY, sP[3] * EY)));
  const double sNY = fma(sP[0], NY, fma(-sP[1], EY, fma(-sP[2], NX, sP[3] * EX)));
  // ... and contracted with their derivatives.  Longitude enters only through
  // the hour angle H: dEX/dH = EXh etc., dEXh/dH = -EX, dEYh/dH = -EY,
  // dNXh/dH = -NX, dNYh/dH = -(NY + clst), dEYt/dH = st cH, dNYt/dH =
  // -st sl sH, d dH/dH = -k1 cH, d dT/dH = -k1t sH.
  const double glon = fma(aEX, EXh, fma(aEY, EYh, fma(aNX, NXh, fma(aNY, NYh,
                      fma(-aEXh, EX, fma(-aEYh, EY, fma(-aNXh, NX, fma(-aNYh, NY + sa.clst,
                      fma(aEYt, sa.st * cH, fma(-aNYt, sa.st * sa.sl * sH,
                      fma(-bdH, sa.k1 * cH, -bdT * sa.k1t * sH)))))))))));
  const double slon = fma(sEX, EXh, fma(sEY, EYh, fma(sNX, NXh, sNY * NYh)));
  // Latitude: sl' = cl, cl' = -sl, so EX, EY, EXh, EYh, EYt do not move,
  // dNX = -cl sH, dNY = sl st - cl ct cH, dNXh = -cl cH, dNYh = cl ct sH,
  // dNYt = st cl cH + sl ct; the delay coefficients k1 = -R cl st,
  // k1t = -R cl ct, k0t = R sl st give d dH = -R sl st sH and
  // d dT = R (sl ct cH + cl st).
  const double cl = sa.cl, sl = sa.sl, ct = sa.ct, st = sa.st;
  const double dNY = fma(sl, st, -cl * ct * cH);
  const double glat = fma(aNX, -cl * sH, fma(aNY, dNY, fma(aNXh, -cl * cH, fma(aNYh, cl * ct * sH,
                      fma(aNYt, fma(st * cl, cH, sl * ct), fma(bdH, -kREarthS * sl * st * sH,
                      bdT * kREarthS * fma(sl * ct, cH, cl * st)))))));
  const double slat = fma(sNX, -cl * sH, sNY * dNY);
  acc[kAdjT + 0] += glat;
  acc[kAdjT + 1] += glon;
  acc[kAdjS + 0] += slat;
  acc[kAdjS + 1] += slon;
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

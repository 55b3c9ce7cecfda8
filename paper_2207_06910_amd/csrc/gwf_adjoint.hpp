// gwf_adjoint.hpp -- per-point mathematics of the adjoint of the Fisher/SNR
// map with respect to the detector parameters (latitude, longitude, arm angle
// gamma and ln S0 of each site).
//
// For a figure of merit J(Gamma_e, SNR_e) the reverse-mode sensitivity
// along a detector parameter xi is
//   dJ/dxi = sum_e [ sum_ij Gbar_e,ij dGamma_e,ij/dxi + snrbar_e dSNR_e/dxi ],
// Gbar = dJ/dGamma (Gamma^-1 for J = ln det Gamma), snrbar = dJ/dSNR.  With
// Gamma_ij = sum_{k,d} w Re(D_i D_j^*) (sec. 3.2, D the noise-weighted
// derivative vectors of the phase-free form) and a symmetric Gbar, each
// grid point and interferometer contributes w (Dr^T Gbar Dr + Di^T Gbar Di)
// to sum_ij Gbar_ij Gamma_ij.  The backward pass recomputes that quadratic
// form at every point and takes its derivatives; no Jacobian is stored.
//
// Structure used (exact algebra).  An interferometer enters D only through
// its six pattern values y = (F+, Fx, dF+/dH, dFx/dH, dF+/dth, dFx/dth)
// (H the hour angle): with c+ = (1 + cos^2 i)/2, cx = cos i,
//   Dr = v0 y0 + (-cx rho + 2 c+ e6) y1 + c+ gamma y2 + c+ e3 y4,
//   Di = (c+ rho - 2 cx e6) y0 + w1 y1 + cx gamma y3 + cx e3 y5,
// where e3, e6 are the unit vectors of theta and psi, v0 and w1 fixed
// per-event vectors (amplitude, distance and inclination rows), gamma the
// hour-angle direction of the phase derivatives (Mc, eta through the
// sidereal angle at t(f); phi; tc) and rho = pi + 2 pi f (dDelta/dH gamma +
// dDelta/dth e3) the site's phase-derivative vector (pi: the PN phase
// derivatives, 2 pi f for tc and the phase-only coefficients c_i).  So the
// form is y^T H y with H = M^T Gbar M built from the Gbar inner products
// <a, b> = a^T Gbar b of just six vectors {pi, gamma, e3, e6, v0, w1}: those
// among the fixed ones once per event, those with pi and gamma once per grid
// point (shared by all sites), and those with rho, which depend on the
// site's arrival-time derivatives, by two multiply-adds each per site.  Per
// interferometer the point then needs two 4 x 4 quadratic forms in y instead
// of z = Gbar D (an 8 x 8 product for two vectors).
//
// Derivatives: J_point depends on the detector parameters through y (the
// patterns: latitude and gamma move their coefficients, longitude the hour
// angle H), through the arrival-time derivatives dDelta/dH and dDelta/dth
// (latitude and longitude) and, for ln S0, through the weight (dw = -w).
// The patterns are trigonometric polynomials in H (SiteC::jk), so along
// longitude y' follows from the same coefficients, and along latitude and
// gamma from their per-event derivatives (AdjSiteC).
#pragma once

#include "gwf_model.hpp"

namespace gwf {

constexpr int kMaxNpi = 6;

// ----------------------------------------------------- site constants
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

// Adds k (a' b + a b') to out: the derivative of trig_mul_add(a, b, k) along
// a direction in which a and b move by a' and b'.
__host__ __device__ inline void trig_mul_add_d(const TrigLin& a, const TrigLin& ad, const TrigLin& b,
                                               const TrigLin& bd, double k, double out[5]) {
  trig_mul_add(ad, b, k, out);
  trig_mul_add(a, bd, k, out);
}

// The latitude derivatives of pattern_trig's polynomials: sin lat -> cos lat,
// cos lat -> -sin lat, which moves only NX, NY and the theta derivative of NY.
__host__ __device__ inline void pattern_trig_lat(double ct, double st, double sl, double cl, double pc[4][5],
                                                 double ptc[4][5]) {
  const TrigLin EX{0.0, 1.0, 0.0}, EY{0.0, 0.0, -ct}, NX{0.0, 0.0, -sl}, NY{-cl * st, -sl * ct, 0.0};
  const TrigLin EYt{0.0, 0.0, st}, NYt{-cl * ct, sl * st, 0.0};
  const TrigLin Z{0.0, 0.0, 0.0};
  const TrigLin NXl{0.0, 0.0, -cl}, NYl{sl * st, -cl * ct, 0.0}, NYtl{sl * ct, cl * st, 0.0};
  for (int i = 0; i < 4; ++i)
    for (int m = 0; m < 5; ++m) pc[i][m] = ptc[i][m] = 0.0;
  // P0 = (EX EX - NX NX - EY EY + NY NY)/2
  trig_mul_add_d(NX, NXl, NX, NXl, -0.5, pc[0]);
  trig_mul_add_d(NY, NYl, NY, NYl, 0.5, pc[0]);
  // P1 = EX NX - EY NY
  trig_mul_add_d(EX, Z, NX, NXl, 1.0, pc[1]);
  trig_mul_add_d(EY, Z, NY, NYl, -1.0, pc[1]);
  // P2 = EX EY - NX NY
  trig_mul_add_d(NX, NXl, NY, NYl, -1.0, pc[2]);
  // P3 = EX NY + NX EY
  trig_mul_add_d(EX, Z, NY, NYl, 1.0, pc[3]);
  trig_mul_add_d(NX, NXl, EY, Z, 1.0, pc[3]);
  // theta derivatives: Pt0 = -EY EYt + NY NYt, Pt1 = -(EYt NY + EY NYt),
  // Pt2 = EX EYt - NX NYt, Pt3 = EX NYt + NX EYt
  trig_mul_add_d(NY, NYl, NYt, NYtl, 1.0, ptc[0]);
  trig_mul_add_d(EYt, Z, NY, NYl, -1.0, ptc[1]);
  trig_mul_add_d(EY, Z, NYt, NYtl, -1.0, ptc[1]);
  trig_mul_add_d(NX, NXl, NYt, NYtl, -1.0, ptc[2]);
  trig_mul_add_d(EX, Z, NYt, NYtl, 1.0, ptc[3]);
  trig_mul_add_d(NX, NXl, EYt, Z, 1.0, ptc[3]);
}

// Per (event, site) constants of the adjoint beside SiteC: the latitude and
// gamma derivatives of the effective interferometers' pattern polynomials
// (SiteC::jk, sqrt(weff) included) and the latitude derivatives of the
// arrival-time coefficients.
struct AdjSiteC {
  double jl[2][4][5];                   // d jk / d latitude
  double jg[2][4][5];                   // d jk / d gamma
  double k1l, k1tl, k0tl;               // d(k1, k1t, k0t)/d latitude
  double pad;
};

// sc: the site's SiteC (site_setup) with the same arm_on.
__host__ __device__ inline void adj_site_setup(const double* p, const SiteDesc& sd, const SiteC& sc,
                                               AdjSiteC& as, uint32_t arm_on = 7u) {
  const double th = p[3], psi = p[6];
  const double c2p = cos(2.0 * psi), s2p = sin(2.0 * psi);
  const double ct = cos(th), st = sin(th), sl = sin(sd.lat), cl = cos(sd.lat);
  as.k1l = kREarthS * sl * st;
  as.k1tl = kREarthS * sl * ct;
  as.k0tl = kREarthS * cl * st;
  as.pad = 0.0;
  // gamma derivatives of the effective interferometers' pattern maps
  double alg[2][4] = {}, beg[2][4] = {};
  if (sd.shape == 1) {
    double ag[3][4], bg[3][4];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double al[4], be[4];
      pattern_map_g(sd.gamma + kPi / 6.0 + kTwoPi * k / 3.0, kPi / 3.0, c2p, s2p, al, be, ag[k], bg[k]);
    }
    if ((arm_on & 7u) == 7u) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        alg[0][j] = ag[0][j] + ag[1][j]; beg[0][j] = bg[0][j] + bg[1][j];
        alg[1][j] = ag[0][j] - ag[1][j]; beg[1][j] = bg[0][j] - bg[1][j];
      }
    } else {                                 // the active arms in arm order
      int m = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (arm_on >> k & 1u) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (m == 0) { alg[0][j] = ag[k][j]; beg[0][j] = bg[k][j]; }
            else { alg[1][j] = ag[k][j]; beg[1][j] = bg[k][j]; }
          }
          ++m;
        }
    }
  } else {
    double al[4], be[4];
    pattern_map_g(sd.gamma, sd.zeta, c2p, s2p, al, be, alg[0], beg[0]);
  }
  // coefficient q of effective interferometer j: sqrt(weff) (a . pm, b . pm,
  // a . ptm, b . ptm) for the maps (a, b) and polynomials (pm, ptm) given
  auto contract = [&](int j, const double (&a)[4], const double (&b)[4], const double (&pm)[4][5],
                      const double (&ptm)[4][5], double (&out)[4][5]) {
    const double w = sqrt(sc.weff[j]);
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      double t[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        t[0] = fma(a[i], pm[i][m], t[0]);
        t[1] = fma(b[i], pm[i][m], t[1]);
        t[2] = fma(a[i], ptm[i][m], t[2]);
        t[3] = fma(b[i], ptm[i][m], t[3]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) out[q][m] = w * t[q];
    }
  };
  {
    double pcl[4][5], ptcl[4][5];
    pattern_trig_lat(ct, st, sl, cl, pcl, ptcl);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) { a[i] = sc.alpha[j][i]; b[i] = sc.beta[j][i]; }
      contract(j, a, b, pcl, ptcl, as.jl[j]);
    }
  }
  {
    double pc[4][5], ptc[4][5];
    pattern_trig(ct, st, sl, cl, pc, ptc);
#pragma unroll
    for (int j = 0; j < 2; ++j) contract(j, alg[j], beg[j], pc, ptc, as.jg[j]);
  }
}

// ----------------------------------------------------- event constants
// The fixed vectors (length P): e3, e6, v0 = (dlnA c+, 0, -c+/dL, 0, 0,
// dc+/di, 0, 0, 0...), w1 = (dlnA cx, 0, -cx/dL, 0, 0, dcx/di, 0, 0, 0...),
// and gamma0 = -e4 + Omega e7 (the part of gamma that does not depend on
// the point).
enum { kXe3 = 0, kXe6, kXv0, kXw1, kXg0, kNX };

__host__ __device__ constexpr int xx_index(int a, int b) {
  return a <= b ? a * kNX - (a * (a - 1)) / 2 + (b - a) : b * kNX - (b * (b - 1)) / 2 + (a - b);
}
__host__ __device__ constexpr int cc_index(int i, int j) {
  return i <= j ? i * kMaxNpi - (i * (i - 1)) / 2 + (j - i) : j * kMaxNpi - (j * (j - 1)) / 2 + (i - j);
}

// Contractions of an event's (symmetrised, masked) Gbar: rows b = Mc, eta,
// tc (the point-dependent basis rows of pi and gamma), the phase-only rows
// 8 + i and the fixed vectors.
struct AdjEventC {
  double g3[6];                              // <e_a, e_b>, (a, b) = 00, 01, 07, 11, 17, 77
  double bx[3][kNX];                         // <e_b, X>, b = Mc, eta, tc
  double cx[kNX][kMaxNpi];                   // <e_{8+i}, X>
  double cb[3][kMaxNpi];                     // <e_b, e_{8+i}>
  double cq[kMaxNpi * (kMaxNpi + 1) / 2];    // <e_{8+i}, e_{8+j}> for i = j, twice that for i < j
  double xx[kNX * (kNX + 1) / 2];            // <X, Y>
  double cpl, ccr;                           // c+, cx
  // products of the above that the per-site rows need (see adjoint_site)
  double h00c, h11c;                         // <v0,v0> + 4 cx^2 <e6,e6>, <w1,w1> + 4 c+^2 <e6,e6>
  double h01c;                               // 2 c+ <e6,v0> - 2 cx <e6,w1>
  double h04, h15;                           // c+ <e3,v0>, cx <e3,w1>
  double cpx33, cxx33;                       // c+ <e3,e3>, cx <e3,e3>
  double cp2x36, cx2x36;                     // 2 c+ <e3,e6>, 2 cx <e3,e6>
  int32_t ok, pad;
};

// gb(i, j): Gbar_ij, symmetric, zero outside the event's rows.  The fixed
// vectors have at most three nonzero entries each, so Gbar X takes those
// columns of Gbar only; every index is fixed at compile time.
template <int NPI, class GB>
__host__ __device__ inline void adj_event_setup(const EventC& ec, const GB& gb, AdjEventC& ae) {
  const double v0a = ec.dlnA_dMc * ec.cplus, v0b = -ec.cplus * ec.inv_dL, v0c = ec.dcplus;
  const double w1a = ec.dlnA_dMc * ec.ccross, w1b = -ec.ccross * ec.inv_dL, w1c = ec.dcross;
  // X_x^T v for a vector v on the binary's eight rows (Mc, eta, dL, theta,
  // phi, iota, psi, tc)
  auto xdot = [&](int x, const double* v) -> double {
    switch (x) {
      case kXe3: return v[3];
      case kXe6: return v[6];
      case kXv0: return fma(v0c, v[5], fma(v0b, v[2], v0a * v[0]));
      case kXw1: return fma(w1c, v[5], fma(w1b, v[2], w1a * v[0]));
      default: return fma(kOmegaE, v[7], -v[4]);
    }
  };
  double GX[kNX][8];                           // (Gbar X)_r on the eight rows
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double row[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) row[c] = gb(r, c);
#pragma unroll
    for (int x = 0; x < kNX; ++x) GX[x][r] = xdot(x, row);
  }
#pragma unroll
  for (int i = 0; i < kMaxNpi; ++i) {
    double row[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) row[c] = i < NPI ? gb(8 + i, c) : 0.0;
#pragma unroll
    for (int x = 0; x < kNX; ++x) ae.cx[x][i] = i < NPI ? xdot(x, row) : 0.0;
  }
  constexpr int rows[3] = {0, 1, 7};
  ae.g3[0] = gb(0, 0); ae.g3[1] = gb(0, 1); ae.g3[2] = gb(0, 7);
  ae.g3[3] = gb(1, 1); ae.g3[4] = gb(1, 7); ae.g3[5] = gb(7, 7);
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int x = 0; x < kNX; ++x) ae.bx[b][x] = GX[x][rows[b]];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int i = 0; i < kMaxNpi; ++i) ae.cb[b][i] = i < NPI ? gb(rows[b], 8 + i) : 0.0;
#pragma unroll
  for (int i = 0; i < kMaxNpi; ++i)
#pragma unroll
    for (int j = i; j < kMaxNpi; ++j)
      ae.cq[cc_index(i, j)] = (i < NPI && j < NPI) ? (i == j ? 1.0 : 2.0) * gb(8 + i, 8 + j) : 0.0;
#pragma unroll
  for (int x = 0; x < kNX; ++x)
#pragma unroll
    for (int y = x; y < kNX; ++y) ae.xx[xx_index(x, y)] = xdot(y, GX[x]);
  ae.cpl = ec.cplus;
  ae.ccr = ec.ccross;
  const double cp = ec.cplus, cx = ec.ccross;
  const double x66 = ae.xx[xx_index(kXe6, kXe6)], x33 = ae.xx[xx_index(kXe3, kXe3)];
  const double x36 = ae.xx[xx_index(kXe3, kXe6)];
  ae.h00c = ae.xx[xx_index(kXv0, kXv0)] + 4.0 * cx * cx * x66;
  ae.h11c = ae.xx[xx_index(kXw1, kXw1)] + 4.0 * cp * cp * x66;
  ae.h01c = 2.0 * cp * ae.xx[xx_index(kXe6, kXv0)] - 2.0 * cx * ae.xx[xx_index(kXe6, kXw1)];
  ae.h04 = cp * ae.xx[xx_index(kXe3, kXv0)];
  ae.h15 = cx * ae.xx[xx_index(kXe3, kXw1)];
  ae.cpx33 = cp * x33;
  ae.cxx33 = cx * x33;
  ae.cp2x36 = 2.0 * cp * x36;
  ae.cx2x36 = 2.0 * cx * x36;
  ae.pad = 0;
}

// Accumulator slots of one site: sum Gbar dGamma along (lat, lon, gamma,
// ln S0), dSNR^2 along (lat, lon, gamma), and SNR^2 itself (its ln S0
// derivative is minus that).
enum { kAdjT = 0, kAdjS = 4, kAdjW = 7, kAdjN = 8 };

// ------------------------------------------------------ one grid point
// The point quantities shared by all sites: the inner products of pi and
// gamma with each other and with the fixed vectors.
struct AdjPoint {
  Point q;
  double pX[kNX];        // <pi, X>
  double gX[4];          // <gamma, X>, X = e3, e6, v0, w1
  double pp, pg, gg;     // <pi, pi>, <pi, gamma>, <gamma, gamma>
  // products the per-site rows take from them
  double cpgg, cxgg, cpg3, cxg3;   // c+ <g,g>, cx <g,g>, c+ <g,e3>, cx <g,e3>
  double h02, h13;                 // c+ <g,v0>, cx <g,w1>
  double cp2g6, cx2g6;             // 2 c+ <g,e6>, 2 cx <g,e6>
};

// vrec: v, 1/v and v^-12.42 at the point (GridWalk), or NULL.
template <int NPI, bool ROT>
__host__ __device__ inline void adjoint_point_setup(const EventC& ec, const AdjEventC& ae, int32_t k,
                                                    AdjPoint& ap, const double* vrec = nullptr) {
  point_setup<true, false, PhaseOnly<NPI>::ecc>(ec, k, true, ROT, ap.q, kPsdF64, vrec);
  const Point& q = ap.q;
  double c[NPI];
  phase_only_coefficients<NPI>(ec, q, c);
  // u_b = <e_b, C>, C = sum c_i e_{8+i}; cCc = <C, C>
  double u[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NPI; ++i) t = fma(ae.cb[b][i], c[i], t);
    u[b] = t;
  }
  // cCc = sum_i c_i (Gbar_ii c_i + 2 sum_{j > i} Gbar_ij c_j)
  double cCc = 0.0;
#pragma unroll
  for (int i = 0; i < NPI; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = i; j < NPI; ++j) t = fma(ae.cq[cc_index(i, j)], c[j], t);
    cCc = fma(c[i], t, cCc);
  }
  // pi = pMc e0 + pEta e1 + tf e7 + C
  const double pm = q.pMc, pe = q.pEta, tf = q.tf;
#pragma unroll
  for (int x = 0; x < kNX; ++x) {
    double t = fma(pm, ae.bx[0][x], fma(pe, ae.bx[1][x], tf * ae.bx[2][x]));
#pragma unroll
    for (int i = 0; i < NPI; ++i) t = fma(c[i], ae.cx[x][i], t);
    ap.pX[x] = t;
  }
  const double pe0 = fma(pm, ae.g3[0], fma(pe, ae.g3[1], fma(tf, ae.g3[2], u[0])));   // <pi, e0>
  const double pe1 = fma(pm, ae.g3[1], fma(pe, ae.g3[3], fma(tf, ae.g3[4], u[1])));   // <pi, e1>
  const double pe7 = fma(pm, ae.g3[2], fma(pe, ae.g3[4], fma(tf, ae.g3[5], u[2])));   // <pi, e7>
  ap.pp = fma(pm, pe0, fma(pe, pe1, fma(tf, pe7, fma(pm, u[0], fma(pe, u[1], fma(tf, u[2], cCc))))));
  // gamma = gMc e0 + gEta e1 + gamma0 (gMc = gEta = 0 without rotation)
  const double gm = q.gMc, ge = q.gEta;
#pragma unroll
  for (int x = 0; x < 4; ++x) ap.gX[x] = fma(gm, ae.bx[0][x], fma(ge, ae.bx[1][x], ae.xx[xx_index(kXg0, x)]));
  ap.pg = fma(gm, pe0, fma(ge, pe1, ap.pX[kXg0]));
  const double ge0 = fma(gm, ae.g3[0], fma(ge, ae.g3[1], 2.0 * ae.bx[0][kXg0]));
  const double ge1 = fma(gm, ae.g3[1], fma(ge, ae.g3[3], 2.0 * ae.bx[1][kXg0]));
  ap.gg = fma(gm, ge0, fma(ge, ge1, ae.xx[xx_index(kXg0, kXg0)]));
  const double cp = ae.cpl, cx = ae.ccr;
  ap.cpgg = cp * ap.gg;
  ap.cxgg = cx * ap.gg;
  ap.cpg3 = cp * ap.gX[kXe3];
  ap.cxg3 = cx * ap.gX[kXe3];
  ap.h02 = cp * ap.gX[kXv0];
  ap.h13 = cx * ap.gX[kXw1];
  ap.cp2g6 = 2.0 * cp * ap.gX[kXe6];
  ap.cx2g6 = 2.0 * cx * ap.gX[kXe6];
}

// A trigonometric polynomial of SiteC::jk and its second hour-angle
// derivative from the same partial sums: with a1 = c1 cos H + c2 sin H and
// a2 = c3 cos 2H + c4 sin 2H, y = c0 + a1 + a2 and y'' = -(a1 + 4 a2).
__host__ __device__ inline void trig_val_dHH(const double c[5], const SiteTrig& sp, double& y, double& yhh) {
  const double a1 = fma(c[2], sp.sH, c[1] * sp.cH);
  const double a2 = fma(c[4], sp.s2H, c[3] * sp.c2H);
  y = (a1 + a2) + c[0];
  yhh = -fma(4.0, a2, a1);
}

// Adds the contribution of one site at the point to acc[kAdjN].
template <bool TAB>
__host__ __device__ inline void adjoint_site(const AdjEventC& ae, const SiteC& sc, const AdjSiteC& as,
                                             const AdjPoint& ap, double* acc) {
  const Point& q = ap.q;
  SiteTrig sp;
  site_trig<false, true, TAB>(sc, q, sp);
  const double tf = q.tf;
  const double a = tf * sp.dH, b = tf * sp.dT;
  const double cp = ae.cpl, cx = ae.ccr;
  // <rho, X> for the site's rho = pi + a gamma + b e3
  double R[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) R[x] = fma(a, ap.gX[x], fma(b, ae.xx[xx_index(kXe3, x)], ap.pX[x]));
  const double Rg = fma(a, ap.gg, fma(b, ap.gX[kXe3], ap.pg));
  const double Rr = fma(a, ap.pg + Rg, fma(b, ap.pX[kXe3] + R[kXe3], ap.pp));   // <rho, rho>
  // rows gamma^T Gbar M and e3^T Gbar M of the real (y0, y1, y2, y4) and
  // imaginary (y0, y1, y3, y5) parts
  const double rg1 = fma(-cx, Rg, ap.cp2g6);
  const double re1 = fma(-cx, R[kXe3], ae.cp2x36);
  const double ig0 = fma(cp, Rg, -ap.cx2g6);
  const double ie0 = fma(cp, R[kXe3], -ae.cx2x36);
  // rows 0 and 1 of Hr + Hi (the y0, y1 rows, where both parts meet)
  const double f = 4.0 * cp * cx * R[kXe6];
  const double h00 = fma(cp * cp, Rr, ae.h00c - f);
  const double h11 = fma(cx * cx, Rr, ae.h11c - f);
  const double h01 = fma(-cx, R[kXv0], fma(cp, R[kXw1], ae.h01c));
  const double h03 = cx * ig0, h05 = cx * ie0, h12 = cp * rg1, h14 = cp * re1;
  const double twom = 2.0 * sp.om;
  const double om = sp.om;
  const double wp = twom * cp, wx = twom * cx;     // 2 w c+, 2 w cx
  double wdH = 0.0, wdT = 0.0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (j >= sc.n_eff) break;
    const double(*C)[5] = sc.jk[j];
    double y0, y1, y2h, y3h;
    trig_val_dHH(C[0], sp, y0, y2h);
    trig_val_dHH(C[1], sp, y1, y3h);
    const double y2 = trig_dH(C[0], sp), y3 = trig_dH(C[1], sp);
    const double y4 = trig_val(C[2], sp), y5 = trig_val(C[3], sp);
    const double tgr = fma(ap.gX[kXv0], y0, fma(rg1, y1, fma(ap.cpgg, y2, ap.cpg3 * y4)));
    const double ter = fma(ae.xx[xx_index(kXe3, kXv0)], y0, fma(re1, y1, fma(ap.cpg3, y2, ae.cpx33 * y4)));
    const double tgi = fma(ig0, y0, fma(ap.gX[kXw1], y1, fma(ap.cxgg, y3, ap.cxg3 * y5)));
    const double tei = fma(ie0, y0, fma(ae.xx[xx_index(kXe3, kXw1)], y1, fma(ap.cxg3, y3, ae.cxx33 * y5)));
    const double hy0 = fma(h00, y0, fma(h01, y1, fma(ap.h02, y2, fma(h03, y3, fma(ae.h04, y4, h05 * y5)))));
    const double hy1 = fma(h01, y0, fma(h11, y1, fma(h12, y2, fma(ap.h13, y3, fma(h14, y4, ae.h15 * y5)))));
    // the point's Gbar-weighted quadratic form, and its gradient in y (times 2 w)
    const double J = fma(y0, hy0, fma(y1, hy1, fma(cp, fma(y2, tgr, y4 * ter), cx * fma(y3, tgi, y5 * tei))));
    const double g0 = twom * hy0, g1 = twom * hy1;
    const double g2 = wp * tgr, g3 = wx * tgi, g4 = wp * ter, g5 = wx * tei;
    // Q = (c+ y0, cx y1); the arrival-time derivatives' adjoints (times 1/tf)
    const double Qr = cp * y0, Qi = cx * y1;
    wdH = fma(twom, fma(Qr, tgi, -Qi * tgr), wdH);
    wdT = fma(twom, fma(Qr, tei, -Qi * ter), wdT);
    // SNR^2 = sum w |Q|^2 and its gradient in (y0, y1)
    const double q2 = fma(Qr, Qr, Qi * Qi);
    const double s0 = wp * Qr, s1 = wx * Qi;
    // longitude (= hour angle): y0' = y2, y1' = y3
    const double y4h = trig_dH(C[2], sp), y5h = trig_dH(C[3], sp);
    acc[kAdjT + 1] = fma(g0, y2, fma(g1, y3, fma(g2, y2h, fma(g3, y3h, fma(g4, y4h, fma(g5, y5h, acc[kAdjT + 1]))))));
    acc[kAdjS + 1] = fma(s0, y2, fma(s1, y3, acc[kAdjS + 1]));
    // latitude
    {
      const double(*L)[5] = as.jl[j];
      const double l0 = trig_val(L[0], sp), l1 = trig_val(L[1], sp);
      const double l2 = trig_dH(L[0], sp), l3 = trig_dH(L[1], sp);
      const double l4 = trig_val(L[2], sp), l5 = trig_val(L[3], sp);
      acc[kAdjT + 0] = fma(g0, l0, fma(g1, l1, fma(g2, l2, fma(g3, l3, fma(g4, l4, fma(g5, l5, acc[kAdjT + 0]))))));
      acc[kAdjS + 0] = fma(s0, l0, fma(s1, l1, acc[kAdjS + 0]));
    }
    // gamma
    {
      const double(*G)[5] = as.jg[j];
      const double l0 = trig_val(G[0], sp), l1 = trig_val(G[1], sp);
      const double l2 = trig_dH(G[0], sp), l3 = trig_dH(G[1], sp);
      const double l4 = trig_val(G[2], sp), l5 = trig_val(G[3], sp);
      acc[kAdjT + 2] = fma(g0, l0, fma(g1, l1, fma(g2, l2, fma(g3, l3, fma(g4, l4, fma(g5, l5, acc[kAdjT + 2]))))));
      acc[kAdjS + 2] = fma(s0, l0, fma(s1, l1, acc[kAdjS + 2]));
    }
    acc[kAdjT + 3] = fma(-om, J, acc[kAdjT + 3]);
    acc[kAdjW] = fma(om, q2, acc[kAdjW]);
  }
  // arrival-time derivatives: dDelta/dH = -k1 sin H, dDelta/dth = k1t cos H + k0t
  //   d/dH:   d(dDelta/dH) = -k1 cos H,      d(dDelta/dth) = -k1t sin H
  //   d/dlat: d(dDelta/dH) = -k1l sin H,     d(dDelta/dth) = k1tl cos H + k0tl
  acc[kAdjT + 1] += tf * fma(wdH, -sc.k1 * sp.cH, -wdT * sc.k1t * sp.sH);
  acc[kAdjT + 0] += tf * fma(wdH, -as.k1l * sp.sH, wdT * fma(as.k1tl, sp.cH, as.k0tl));
}

// One grid point and one site (host checks).
template <int NPI, bool ROT>
__host__ __device__ inline void adjoint_point(const EventC& ec, const AdjEventC& ae, const SiteC& sc,
                                              const AdjSiteC& as, int32_t k, double* acc) {
  AdjPoint ap;
  adjoint_point_setup<NPI, ROT>(ec, ae, k, ap);
  adjoint_site<true>(ae, sc, as, ap, acc);
}

}  // namespace gwf

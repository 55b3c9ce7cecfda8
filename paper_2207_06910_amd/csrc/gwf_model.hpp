// gwf_model.hpp -- per-event, per-site and per-frequency mathematics of the
// Fisher/SNR path, shared by the HIP kernels of libgwf.
//
// The strain at interferometer i is h_i = A(f) Q_i(f) exp(i Psi_i(f)) with
//   A      restricted (Newtonian) amplitude, |h~| = sqrt(5/24) pi^{-2/3}
//          (G Mc/c^3)^{5/6} f^{-7/6} c/dL                          (sec. 2.2)
//   Q_i    F+_i (1+cos^2 iota)/2 + i Fx_i cos iota, the pattern-weighted
//          polarisations (sec. 3.1, GWAmplitudes)
//   Psi_i  2 pi f (tc + Delta_i) - Phic - pi/4 + Psi_PN, with Delta_i the
//          arrival-time offset of the site (Doppler term of the Earth-motion
//          footnote of sec. 3) and Psi_PN the TaylorF2 phase (sec. 2.2).
// Patterns and Delta_i are evaluated at the sidereal angle of t(f) = tc -
// tau*(f) when the Earth rotates (sec. 2.2, tau_star).
//
// Because every product entering SNR^2 and the Fisher matrix has the form
// d_a h d_b h^*, the common factor exp(i Psi_i) cancels:
//   d_a h_i = A (D_a + ...) exp(i Psi_i),  D_a = d_a Q_i + Q_i d_a ln A + i Q_i d_a Psi_i,
// so no sine or cosine of the (large) phase is ever needed here, only its
// derivatives.  Those of the PN phase are polynomials in v = (pi G M f/c^3)^{1/3}
// and ln v whose per-event coefficients are built once (PhaseSeries).
//
// Antenna patterns are written in closed form in the hour angle H of the
// source at the site: with E, N the local East/North unit vectors and the
// polarisation frame (e_phi, e_theta) of the source,
//   EX = E.e_phi = cos H,           EY = E.e_theta = -cos th sin H,
//   NX = N.e_phi = -sin lat sin H,  NY = N.e_theta = -sin lat cos th cos H - cos lat sin th,
// the detector tensor (sin zeta/2)[sin 2g (EE-NN) - cos 2g (EN+NE)] gives
//   F+ = sin z [a cos 2psi + b sin 2psi],  Fx = sin z [b cos 2psi - a sin 2psi],
//   a = sin2g P1 - cos2g P2,  b = sin2g P3 - cos2g P4,
//   P1 = (EX^2 - NX^2 - EY^2 + NY^2)/2, P2 = EX NX - EY NY,
//   P3 = EX EY - NX NY,  P4 = EX NY + NX EY,
// a derivation of this library (equivalent to the tensor contraction).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "gwf_arith.hpp"

namespace gwf {

// ----------------------------------------------------------- constants
// IAU 2015 nominal values (the paper fixes none numerically).
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 2.0 * kPi;
constexpr double kC = 299792458.0;
constexpr double kGMsun = 1.3271244e20;
constexpr double kTsun = kGMsun / (kC * kC * kC);           // s
constexpr double kAU = 149597870700.0;
constexpr double kPc = kAU * 648000.0 / kPi;                 // m
constexpr double kGpcS = 1e9 * kPc / kC;                     // s
constexpr double kSiderealDay = 86164.0905;                  // s
constexpr double kOmegaE = kTwoPi / kSiderealDay;            // rad/s
constexpr double kREarthS = 6.371e6 / kC;                    // s
constexpr double kEulerGamma = 0.5772156649015329;
constexpr double kLn2 = 0.69314718055994530942;

constexpr int kMaxSites = 8;
constexpr int kMaxPar = 14;     // Fisher rows with tides and eccentricity
constexpr int kMaxIfo = 16;
constexpr uint32_t kFlagRot = 1;
constexpr uint32_t kFlagTidal = 2;
constexpr uint32_t kFlagMixed = 4;
constexpr uint32_t kFlagEcc = 8;
constexpr int kNparIn = 15;      // event inputs: the 13 parameters, e0, f_ref (0: the grid start)

enum : int32_t { kEvInvalid = 1, kEvNotPD = 2, kEvIllCond = 4, kEvNonFinite = 8, kEvSkipped = 16, kEvSvd = 32 };

// ------------------------------------------------------------ series
// Per-event coefficients of a PN-phase derivative:
//   s(v) = v^-5 (c0 + c1 v + ... + c7 v^7) + ln v (l5 + l6 v) + v^5 (t10 + t12 v^2)
struct PhaseSeries {
  double c[8];
  double l5, l6, t10, t12;
};
// Per-event coefficients of a tau*-type series:
//   s(v) = v^-8 (c0 + c1 v + ... + c7 v^7) + l6 ln v v^-2
struct TauSeries {
  double c[8];
  double l6;
};

// Index of the phase-derivative series in EventC::ps.
enum { kPsMc = 0, kPsEta, kPsChi1, kPsChi2, kPsL1, kPsL2 };
// Index of the tau-type series in EventC::ts: the rotation angle offset
// -Omega tau*, and the derivatives of the sidereal angle w.r.t. Mc and eta.
enum { kTsTheta = 0, kTsMc, kTsEta };

struct EventC {
  // grid: v_k = exp(lnv0 + k dlnv), f_k = v_k^3 / (pi M), trapezoid weights
  double lnv0, dlnv, inv_piM, piM, wint, wfirst, wlast;
  // sqrt(w KA4 / (pi M)) for the three weights: sqrt(4 w_k A_k^2) = rw v_k^-2
  // (the Fisher kernels' root weight), and a pad that keeps the 16-byte
  // alignment of the fields below, which kernels holding the struct in LDS
  // read in 16-byte pairs
  double rwint, rwfirst, rwlast, pad_rw;
  // explicit grid: the event's frequencies (NULL on a log grid) and ln(pi M),
  // v_k = exp((ln(pi M) + ln f_k)/3), weights (f_{k+1} - f_{k-1})/2
  const double* fx;
  double lnpiM;
  int32_t n;
  int32_t status;
  // amplitude: A^2 = KA v^-7 (factor 4 of the inner product included)
  double KA4;
  double dlnA_dMc, inv_dL;
  // sky/orientation
  double thc;                  // sidereal angle at coalescence, 2 pi tcoal
  double cplus, ccross, dcplus, dcross;   // (1+cos^2 i)/2, cos i and d/d iota
  // their products in the per-point rows of iota, psi and the SNR density:
  // c+^2, cx^2, c+ dcx - cx dc+, -2 c+ cx
  double cp2, cx2, u_iota, u_psi;
  PhaseSeries ps[6];
  TauSeries ts[3];
  // waveform only: Psi_PN / (2 pi) in cycles, ln of the amplitude factor
  // (A = exp(lnA - 3.5 ln v)), and -(Phic + pi/4)/(2 pi)
  PhaseSeries cyc;
  double lnA, cyc0;
  // moderate eccentricity (ecc != 0): the phase gains ecc_psi v^-5 r with
  // r = (v_ref/v)^{19/3} = exp((19/3)(ecc_lnvr - ln v)); ecc_mc v^-5 r joins
  // dPsi/dMc and ecc_e0 v^-5 r is dPsi/de0 (eta does not enter at fixed Mc)
  double ecc_lnvr, ecc_psi, ecc_mc, ecc_e0, ecc_cyc;
  int32_t ecc, pad_ecc;
};

struct SiteC {
  double cdl, sdl;             // cos, sin of (site longitude - phi)
  double ct, slct, clst, sl, st;   // cos th, sin lat cos th, cos lat sin th, sin lat, sin th
  double cl;                   // cos lat
  double k1, k0, k1t, k0t;     // Delta = k1 cos H + k0;  dDelta/dth = k1t cos H + k0t
  double lnx_off, ix_fac, x_fac;  // ln(f/f0) = 3 ln v + lnx_off; f0/f = ix_fac v^-3; f/f0 = x_fac v^3
  double xp_fac;               // (f/f0)^-4.14 = xp_fac v^-12.42
  double S0inv;                // 1/S0
  // S0 times the PSD shape's coefficients (the root weight's form, see
  // psd_root_weight), and sqrt(1/S0)
  double xpS0, m5S0, k111S0, rS0inv;
  double alpha[2][4], beta[2][4], weff[2];  // effective interferometers (pattern maps)
  // the effective interferometers' F+, Fx and their theta derivatives as
  // trigonometric polynomials in the hour angle H: coefficients of
  // (1, cos H, sin H, cos 2H, sin 2H), each scaled by sqrt(weff)
  double jk[2][4][5];
  double arm_alpha[3][4], arm_beta[3][4];   // individual arms (SNR per interferometer)
  int32_t n_eff, n_arm;
  // sampled noise curve (tab_kind 1: PSD, 2: ASD; 0: the analytic PSD above)
  const double* tab_f;
  const double* tab_S;
  int64_t tab_n;
  int32_t tab_kind, pad;
};

// Site description as passed at the boundary (radians); psd_kind 0 is the
// analytic PSD (S0, f0), 1 and 2 a sampled PSD or ASD (tab_f, tab_S,
// tab_n, scaled by S0).
struct SiteDesc {
  double lat, lon, gamma, zeta, S0, f0;
  int32_t shape, psd_kind;
  const double* tab_f;
  const double* tab_S;
  int64_t tab_n;
};

struct NetDesc {
  SiteDesc site[kMaxSites];
  int32_t n_site, n_ifo;
};

// Whether any site of the network has a sampled noise curve (the kernels
// without one leave the check out).
__host__ __device__ inline bool net_has_tables(const NetDesc& nd) {
  for (int s = 0; s < nd.n_site; ++s)
    if (nd.site[s].psd_kind != 0) return true;
  return false;
}

// ------------------------------------------------ per-event coefficients
// Coefficients a_k (k = 0..7), b_5, b_6 (ln v parts) and tidal a_10, a_12 of
// the TaylorF2 phase Psi_PN = 3/(128 eta) v^-5 sum_k (a_k + b_k ln v) v^k,
// together with their partial derivatives with respect to eta (at fixed
// component spins and deformabilities), chi_s, chi_a, Lambda1, Lambda2.
// Point-particle terms to 3.5PN, aligned-spin spin-orbit terms to 3.5PN and
// 2PN spin-spin terms, tidal terms at 5PN/6PN through the combinations of
// eq. (LamTdelLam_def) (refs. of sec. 2.2).
struct PNCoef {
  double a[8], ae[8], as[8], aa[8];   // value, d/deta, d/dchi_s, d/dchi_a
  double b5, b5e, b5s, b5a, b6;
  double a10, a10e, a10_1, a10_2, a12, a12e, a12_1, a12_2;
};

__host__ __device__ inline void pn_coefficients(double eta, double chi1, double chi2, double L1,
                                                double L2, bool tidal, PNCoef& p) {
  const double pi = kPi, pi2 = kPi * kPi;
  const double e2 = eta * eta, e3 = e2 * eta;
  const double dl = sqrt(1.0 - 4.0 * eta);
  const double ddl = -2.0 / dl;     // d delta / d eta
  const double xs = 0.5 * (chi1 + chi2), xa = 0.5 * (chi1 - chi2);
  for (int k = 0; k < 8; ++k) { p.a[k] = 0.0; p.ae[k] = 0.0; p.as[k] = 0.0; p.aa[k] = 0.0; }
  p.a[0] = 1.0;
  // 1PN
  p.a[2] = 3715.0 / 756.0 + (55.0 / 9.0) * eta;
  p.ae[2] = 55.0 / 9.0;
  // 1.5PN: tail and spin-orbit
  p.a[3] = -16.0 * pi + (113.0 / 3.0) * dl * xa + (113.0 / 3.0 - (76.0 / 3.0) * eta) * xs;
  p.ae[3] = (113.0 / 3.0) * ddl * xa - (76.0 / 3.0) * xs;
  p.as[3] = 113.0 / 3.0 - (76.0 / 3.0) * eta;
  p.aa[3] = (113.0 / 3.0) * dl;
  // 2PN: point particle and spin-spin
  p.a[4] = 15293365.0 / 508032.0 + (27145.0 / 504.0) * eta + (3085.0 / 72.0) * e2 +
           (-405.0 / 8.0 + 200.0 * eta) * xa * xa - (405.0 / 4.0) * dl * xa * xs +
           (-405.0 / 8.0 + 2.5 * eta) * xs * xs;
  p.ae[4] = 27145.0 / 504.0 + (3085.0 / 36.0) * eta + 200.0 * xa * xa -
            (405.0 / 4.0) * ddl * xa * xs + 2.5 * xs * xs;
  p.as[4] = -(405.0 / 4.0) * dl * xa + 2.0 * (-405.0 / 8.0 + 2.5 * eta) * xs;
  p.aa[4] = 2.0 * (-405.0 / 8.0 + 200.0 * eta) * xa - (405.0 / 4.0) * dl * xs;
  // 2.5PN: X5 (1 + 3 ln v)
  const double q5 = 732985.0 / 2268.0 + (140.0 / 9.0) * eta;
  const double r5 = -732985.0 / 2268.0 + (24260.0 / 81.0) * eta + (340.0 / 9.0) * e2;
  const double X5 = pi * (38645.0 / 756.0 - (65.0 / 9.0) * eta) - q5 * dl * xa + r5 * xs;
  const double X5e = -(65.0 / 9.0) * pi - (140.0 / 9.0) * dl * xa - q5 * ddl * xa +
                     (24260.0 / 81.0 + (680.0 / 9.0) * eta) * xs;
  const double X5s = r5;
  const double X5a = -q5 * dl;
  p.a[5] = X5; p.ae[5] = X5e; p.as[5] = X5s; p.aa[5] = X5a;
  p.b5 = 3.0 * X5; p.b5e = 3.0 * X5e; p.b5s = 3.0 * X5s; p.b5a = 3.0 * X5a;
  // 3PN: Y6 - (6848/21) ln(4 v)
  const double Y6 = 11583231236531.0 / 4694215680.0 - (640.0 / 3.0) * pi2 -
                    (6848.0 / 21.0) * kEulerGamma +
                    (-15737765635.0 / 3048192.0 + (2255.0 / 12.0) * pi2) * eta +
                    (76055.0 / 1728.0) * e2 - (127825.0 / 1296.0) * e3 +
                    pi * ((2270.0 / 3.0) * dl * xa + (2270.0 / 3.0 - 520.0 * eta) * xs);
  const double Y6e = (-15737765635.0 / 3048192.0 + (2255.0 / 12.0) * pi2) +
                     (76055.0 / 864.0) * eta - (127825.0 / 432.0) * e2 +
                     pi * ((2270.0 / 3.0) * ddl * xa - 520.0 * xs);
  p.a[6] = Y6 - (6848.0 / 21.0) * (2.0 * kLn2);
  p.ae[6] = Y6e;
  p.as[6] = pi * (2270.0 / 3.0 - 520.0 * eta);
  p.aa[6] = pi * (2270.0 / 3.0) * dl;
  p.b6 = -6848.0 / 21.0;
  // 3.5PN
  const double u7 = -25150083775.0 / 3048192.0 + (26804935.0 / 6048.0) * eta - (1985.0 / 48.0) * e2;
  const double w7 = -25150083775.0 / 3048192.0 + (10566655595.0 / 762048.0) * eta -
                    (1042165.0 / 3024.0) * e2 + (5345.0 / 36.0) * e3;
  p.a[7] = pi * (77096675.0 / 254016.0 + (378515.0 / 1512.0) * eta - (74045.0 / 756.0) * e2) +
           u7 * dl * xa + w7 * xs;
  p.ae[7] = pi * (378515.0 / 1512.0 - (74045.0 / 378.0) * eta) +
            (26804935.0 / 6048.0 - (1985.0 / 24.0) * eta) * dl * xa + u7 * ddl * xa +
            (10566655595.0 / 762048.0 - (1042165.0 / 1512.0) * eta + (5345.0 / 12.0) * e2) * xs;
  p.as[7] = w7;
  p.aa[7] = u7 * dl;
  // tides: a10 = -(39/2) Lt, a12 = -(3115/64) Lt + (6595/364) delta dLt
  p.a10 = p.a10e = p.a10_1 = p.a10_2 = 0.0;
  p.a12 = p.a12e = p.a12_1 = p.a12_2 = 0.0;
  if (tidal) {
    const double s = L1 + L2, d = L1 - L2;
    const double q1 = 1.0 + 7.0 * eta - 31.0 * e2, q1e = 7.0 - 62.0 * eta;
    const double q2 = 1.0 + 9.0 * eta - 11.0 * e2, q2e = 9.0 - 22.0 * eta;
    const double Lt = (8.0 / 13.0) * (q1 * s + dl * q2 * d);
    const double Lte = (8.0 / 13.0) * (q1e * s + (ddl * q2 + dl * q2e) * d);
    const double Lt1 = (8.0 / 13.0) * (q1 + dl * q2), Lt2 = (8.0 / 13.0) * (q1 - dl * q2);
    const double r1 = 1.0 - (13272.0 / 1319.0) * eta + (8944.0 / 1319.0) * e2;
    const double r1e = -13272.0 / 1319.0 + (17888.0 / 1319.0) * eta;
    const double r2 = 1.0 - (15910.0 / 1319.0) * eta + (32850.0 / 1319.0) * e2 + (3380.0 / 1319.0) * e3;
    const double r2e = -15910.0 / 1319.0 + (65700.0 / 1319.0) * eta + (10140.0 / 1319.0) * e2;
    const double dLt = 0.5 * (dl * r1 * s + r2 * d);
    const double dLte = 0.5 * ((ddl * r1 + dl * r1e) * s + r2e * d);
    const double dLt1 = 0.5 * (dl * r1 + r2), dLt2 = 0.5 * (dl * r1 - r2);
    p.a10 = -19.5 * Lt; p.a10e = -19.5 * Lte; p.a10_1 = -19.5 * Lt1; p.a10_2 = -19.5 * Lt2;
    const double k12 = 6595.0 / 364.0;
    p.a12 = -(3115.0 / 64.0) * Lt + k12 * dl * dLt;
    p.a12e = -(3115.0 / 64.0) * Lte + k12 * (ddl * dLt + dl * dLte);
    p.a12_1 = -(3115.0 / 64.0) * Lt1 + k12 * dl * dLt1;
    p.a12_2 = -(3115.0 / 64.0) * Lt2 + k12 * dl * dLt2;
  }
}

// tau*(f) = 5 M/(256 eta) v^-8 sum_k (t_k + l_k ln v) v^k at 3.5PN, non-spinning
// (the paper cites Buonanno et al. 2009, eq. 3.8b); t_k and d t_k/d eta.
__host__ __device__ inline void tau_coefficients(double eta, double t[8], double te[8], double& l6) {
  const double pi = kPi, pi2 = kPi * kPi, e2 = eta * eta, e3 = e2 * eta;
  for (int k = 0; k < 8; ++k) { t[k] = 0.0; te[k] = 0.0; }
  t[0] = 1.0;
  t[2] = 743.0 / 252.0 + (11.0 / 3.0) * eta;               te[2] = 11.0 / 3.0;
  t[3] = -32.0 * pi / 5.0;
  t[4] = 3058673.0 / 508032.0 + (5429.0 / 504.0) * eta + (617.0 / 72.0) * e2;
  te[4] = 5429.0 / 504.0 + (617.0 / 36.0) * eta;
  t[5] = pi * (-7729.0 / 252.0 + (13.0 / 3.0) * eta);     te[5] = pi * 13.0 / 3.0;
  // (3424/105) ln(16 v^2) = (3424/105) (4 ln 2 + 2 ln v)
  t[6] = -10052469856691.0 / 23471078400.0 + (128.0 / 3.0) * pi2 + (6848.0 / 105.0) * kEulerGamma +
         (3147553127.0 / 3048192.0 - (451.0 / 12.0) * pi2) * eta - (15211.0 / 1728.0) * e2 +
         (25565.0 / 1296.0) * e3 + (3424.0 / 105.0) * 4.0 * kLn2;
  te[6] = (3147553127.0 / 3048192.0 - (451.0 / 12.0) * pi2) - (15211.0 / 864.0) * eta +
          (25565.0 / 432.0) * e2;
  t[7] = pi * (-15419335.0 / 127008.0 - (75703.0 / 756.0) * eta + (14809.0 / 378.0) * e2);
  te[7] = pi * (-75703.0 / 756.0 + (14809.0 / 189.0) * eta);
  l6 = 2.0 * 3424.0 / 105.0;
}

// Cut frequency: twice the ISCO orbital frequency, 1/(6^{3/2} pi G M/c^3)
// (sec. 2.2 footnote).
__host__ __device__ inline double cut_frequency_of(double M_s) {
  return 1.0 / (6.0 * sqrt(6.0) * kPi * M_s);
}

// x is neither infinite nor NaN (x - x is 0 exactly for finite x).
__host__ __device__ inline bool finite(double x) { return (x - x) == 0.0; }


// Rows of event e's Fisher matrix (bit r: row r; NULL: every row).
__host__ __device__ inline uint32_t event_rows(const uint32_t* par_mask, int64_t e) {
  return par_mask ? par_mask[e] : ~0u;
}

__host__ __device__ inline bool rows_in(uint32_t m, int r, int c) { return ((m >> r) & (m >> c) & 1u) != 0; }

// Parameter validity; returns the status bits of an event.
__host__ __device__ inline int32_t check_event(const double* p, bool tidal, double fmin, double fmax,
                                               int32_t n, bool ecc = false) {
  int32_t st = 0;
  const int np = tidal ? 13 : 11;
  for (int i = 0; i < np; ++i)
    if (!finite(p[i])) st |= kEvNonFinite;
  if (ecc && (!finite(p[13]) || !finite(p[14]))) st |= kEvNonFinite;
  if (!finite(fmin) || !finite(fmax)) st |= kEvNonFinite;
  if (st) return st;
  if (!(p[0] > 0.0) || !(p[1] > 0.0) || !(p[1] <= 0.25) || !(p[2] > 0.0)) st |= kEvInvalid;
  if (fabs(p[9]) > 1.0 || fabs(p[10]) > 1.0) st |= kEvInvalid;
  if (tidal && (p[11] < 0.0 || p[12] < 0.0)) st |= kEvInvalid;
  if (n < 2 || !(fmin > 0.0) || !(fmax > fmin)) st |= kEvInvalid;
  if (ecc && (!(p[13] >= 0.0) || !(p[13] < 1.0) || p[14] < 0.0)) st |= kEvInvalid;
  return st;
}

// Build the per-event constants.  p[13] are the parameters in boundary
// order; fmax <= 0 selects the cut frequency.
// The binary's total mass in seconds, M = Mc eta^(-3/5) G/c^3 (pi M sets the
// grid's v = (pi M f)^(1/3) and the PSD's x = f/f0 of every site).
__host__ __device__ inline double total_mass_s(const double* p) { return p[0] * pow(p[1], -0.6) * kTsun; }

__host__ __device__ inline void event_setup(const double* p, double fmin, double fmax, int32_t n,
                                            uint32_t flags, EventC& ec) {
  const bool tidal = (flags & kFlagTidal) != 0;
  const bool rot = (flags & kFlagRot) != 0;
  const bool ecc = (flags & kFlagEcc) != 0;
  const double Mc = p[0], eta = p[1], dL = p[2];
  const double Ms = total_mass_s(p);
  if (!(fmax > 0.0)) fmax = cut_frequency_of(Ms);
  ec.n = n;
  ec.fx = nullptr;
  ec.ecc = 0;
  ec.ecc_lnvr = ec.ecc_psi = ec.ecc_mc = ec.ecc_e0 = ec.ecc_cyc = 0.0;
  ec.status = check_event(p, tidal, fmin, fmax, n, ecc);
  if (ec.status) return;
  // grid
  const double D = log(fmax / fmin) / (double)(n - 1);
  ec.piM = kPi * Ms;
  ec.inv_piM = 1.0 / ec.piM;
  ec.lnpiM = log(ec.piM);
  ec.lnv0 = (ec.lnpiM + log(fmin)) / 3.0;
  ec.dlnv = D / 3.0;
  ec.wint = sinh(D);                  // interior weight / f_k
  ec.wfirst = 0.5 * expm1(D);         // (f_1 - f_0)/2 / f_0
  ec.wlast = -0.5 * expm1(-D);        // (f_{n-1} - f_{n-2})/2 / f_{n-1}
  // amplitude: 4 A^2 = 4 (5/24) pi^{-4/3} (G Mc/c^3)^{5/3} f^{-7/3} (c/dL)^2, f^{-7/3} = (pi M)^{7/3} v^{-7}
  const double Mcs = Mc * kTsun, dLs = dL * kGpcS;
  ec.KA4 = 4.0 * (5.0 / 24.0) * pow(kPi, -4.0 / 3.0) * pow(Mcs, 5.0 / 3.0) * pow(ec.piM, 7.0 / 3.0) /
           (dLs * dLs);
  ec.rwint = sqrt(ec.wint * ec.KA4 * ec.inv_piM);
  ec.rwfirst = sqrt(ec.wfirst * ec.KA4 * ec.inv_piM);
  ec.rwlast = sqrt(ec.wlast * ec.KA4 * ec.inv_piM);
  ec.pad_rw = 0.0;
  ec.dlnA_dMc = 5.0 / (6.0 * Mc);
  ec.inv_dL = 1.0 / dL;
  // 2 pi tcoal reduced to [0, 2 pi)
  const double tfrac = p[7] - floor(p[7]);
  ec.thc = kTwoPi * tfrac;
  const double ci = cos(p[5]), si = sin(p[5]);
  ec.cplus = 0.5 * (1.0 + ci * ci);
  ec.ccross = ci;
  ec.dcplus = -ci * si;
  ec.dcross = -si;
  ec.cp2 = ec.cplus * ec.cplus;
  ec.cx2 = ec.ccross * ec.ccross;
  ec.u_iota = ec.cplus * ec.dcross - ec.ccross * ec.dcplus;
  ec.u_psi = -2.0 * ec.cplus * ec.ccross;

  // ---- moderate eccentricity (sec. 2.2, is_eccentric): the leading-order
  // correction -(2355/1462) e0^2 (v_ref/v)^{19/3} relative to the Newtonian
  // phase 3/(128 eta v^5) (the model the paper cites, Moore et al. 2016),
  // e0 given where the GW frequency is f_ref (the grid's first frequency
  // unless given, sec. 2.1).  At fixed f and f_ref it is proportional to
  // eta^-1 v^-5, i.e. to Mc^{-5/3} alone.
  if (ecc) {
    const double e0 = p[13], fref = p[14] > 0.0 ? p[14] : fmin;
    const double K = (3.0 / (128.0 * eta)) * (-2355.0 / 1462.0);
    ec.ecc = 1;
    ec.ecc_lnvr = (ec.lnpiM + log(fref)) / 3.0;
    ec.ecc_psi = K * e0 * e0;
    ec.ecc_mc = -5.0 / (3.0 * Mc) * ec.ecc_psi;
    ec.ecc_e0 = 2.0 * K * e0;
    ec.ecc_cyc = ec.ecc_psi / kTwoPi;
  }

  // ---- phase-derivative series
  PNCoef c;
  pn_coefficients(eta, p[9], p[10], tidal ? p[11] : 0.0, tidal ? p[12] : 0.0, tidal, c);
  const double A = 3.0 / (128.0 * eta);
  double b[8] = {0, 0, 0, 0, 0, c.b5, c.b6, 0};
  double be[8] = {0, 0, 0, 0, 0, c.b5e, 0.0, 0};
  // d Psi/d Mc = (1/(3 Mc)) v dPsi/dv
  {
    PhaseSeries& s = ec.ps[kPsMc];
    const double K = A / (3.0 * Mc);
    for (int k = 0; k < 8; ++k) s.c[k] = K * ((k - 5) * c.a[k] + b[k]);
    s.l5 = 0.0;
    s.l6 = K * c.b6;
    s.t10 = K * 5.0 * c.a10;
    s.t12 = K * 7.0 * c.a12;
  }
  // d Psi/d eta = explicit eta dependence - (1/(5 eta)) v dPsi/dv (v ~ eta^{-1/5})
  {
    PhaseSeries& s = ec.ps[kPsEta];
    const double K = A / (5.0 * eta);
    for (int k = 0; k < 8; ++k) s.c[k] = A * (c.ae[k] - c.a[k] / eta) - K * ((k - 5) * c.a[k] + b[k]);
    s.c[0] = 0.0;   // the leading term does not depend on eta at fixed Mc
    s.l5 = A * (be[5] - b[5] / eta);
    s.l6 = A * (-c.b6 / eta) - K * c.b6;
    s.t10 = A * (c.a10e - c.a10 / eta) - K * 5.0 * c.a10;
    s.t12 = A * (c.a12e - c.a12 / eta) - K * 7.0 * c.a12;
  }
  // spins: d/dchi1 = (d/dchi_s + d/dchi_a)/2, d/dchi2 = (d/dchi_s - d/dchi_a)/2
  for (int j = 0; j < 2; ++j) {
    PhaseSeries& s = ec.ps[kPsChi1 + j];
    const double sg = j == 0 ? 1.0 : -1.0;
    for (int k = 0; k < 8; ++k) s.c[k] = 0.5 * A * (c.as[k] + sg * c.aa[k]);
    s.l5 = 0.5 * A * (c.b5s + sg * c.b5a);
    s.l6 = 0.0;
    s.t10 = 0.0;
    s.t12 = 0.0;
  }
  // tides
  for (int j = 0; j < 2; ++j) {
    PhaseSeries& s = ec.ps[kPsL1 + j];
    for (int k = 0; k < 8; ++k) s.c[k] = 0.0;
    s.l5 = s.l6 = 0.0;
    s.t10 = A * (j == 0 ? c.a10_1 : c.a10_2);
    s.t12 = A * (j == 0 ? c.a12_1 : c.a12_2);
  }

  // Psi_PN itself, in cycles, for the strain output
  {
    PhaseSeries& s = ec.cyc;
    const double K = A / kTwoPi;
    for (int k = 0; k < 8; ++k) s.c[k] = K * c.a[k];
    s.l5 = K * c.b5;
    s.l6 = K * c.b6;
    s.t10 = K * c.a10;
    s.t12 = K * c.a12;
  }
  ec.lnA = 0.5 * log(0.25 * ec.KA4);
  ec.cyc0 = -(p[8] + 0.25 * kPi) / kTwoPi;

  // ---- rotation: sidereal-angle offset -Omega tau* and its Mc, eta derivatives
  double t[8], te[8], l6;
  tau_coefficients(eta, t, te, l6);
  const double Kt = 5.0 * Ms / (256.0 * eta);
  const double om = rot ? kOmegaE : 0.0;
  double lk[8] = {0, 0, 0, 0, 0, 0, l6, 0};
  for (int k = 0; k < 8; ++k) {
    ec.ts[kTsTheta].c[k] = -om * Kt * t[k];
    // d tau*/d Mc = (Kt/Mc) sum [(t_k + l_k L)(1 + (k-8)/3) + l_k/3] v^(k-8)
    ec.ts[kTsMc].c[k] = -om * (Kt / Mc) * ((1.0 + (k - 8) / 3.0) * t[k] + lk[k] / 3.0);
    // d tau*/d eta = Kt sum [t_k' - (k t_k + l_k)/(5 eta)] v^(k-8) + log part
    ec.ts[kTsEta].c[k] = -om * Kt * (te[k] - (k * t[k] + lk[k]) / (5.0 * eta));
  }
  ec.ts[kTsEta].c[0] = 0.0;   // leading tau* does not depend on eta at fixed Mc
  ec.ts[kTsTheta].l6 = -om * Kt * l6;
  ec.ts[kTsMc].l6 = -om * (Kt / Mc) * (1.0 + (6 - 8) / 3.0) * l6;
  ec.ts[kTsEta].l6 = -om * Kt * (-6.0 * l6 / (5.0 * eta));
}

// event_setup on event e's grid: the log descriptors, or an explicit grid
// (gf non-NULL; event e's npts[e] frequencies from gf + goff[e]) bounded by
// its first and last frequency, which must be positive and increasing (the
// event is flagged invalid otherwise, before any other frequency is read).
__host__ __device__ inline void event_setup_grid(const double* p, const double* fmin, const double* fmax,
                                                 const int32_t* npts, const int64_t* goff, const double* gf,
                                                 int64_t e, uint32_t flags, EventC& ec) {
  const int32_t n = npts[e];
  if (gf) {
    const double* fx = gf + goff[e];
    const bool ok = n >= 2 && fx[0] > 0.0 && fx[n - 1] > fx[0];
    event_setup(p, ok ? fx[0] : 0.0, ok ? fx[n - 1] : 0.0, n, flags, ec);
    ec.fx = fx;
  } else {
    event_setup(p, fmin[e], fmax ? fmax[e] : 0.0, n, flags, ec);
  }
}

// A function u + v cos H + w sin H of the hour angle H.
struct TrigLin {
  double u, v, w;
};

// Adds k a b to out, the coefficients of (1, cos H, sin H, cos 2H, sin 2H).
__host__ __device__ inline void trig_mul_add(const TrigLin& a, const TrigLin& b, double k, double out[5]) {
  out[0] += k * fma(a.u, b.u, 0.5 * fma(a.v, b.v, a.w * b.w));
  out[1] += k * fma(a.u, b.v, a.v * b.u);
  out[2] += k * fma(a.u, b.w, a.w * b.u);
  out[3] += k * 0.5 * fma(a.v, b.v, -a.w * b.w);
  out[4] += k * 0.5 * fma(a.v, b.w, a.w * b.v);
}

// The pattern vector P(H) of site_point and its theta derivative as
// trigonometric polynomials of degree two in the hour angle: the frame
// components EX = cos H, EY = -cos th sin H, NX = -sin lat sin H,
// NY = -(sin lat cos th cos H + cos lat sin th) are linear in (cos H, sin H),
// and every component of P is a quadratic form in them.
__host__ __device__ inline void pattern_trig(double ct, double st, double sl, double cl, double pc[4][5],
                                             double ptc[4][5]) {
  const TrigLin EX{0.0, 1.0, 0.0}, EY{0.0, 0.0, -ct}, NX{0.0, 0.0, -sl}, NY{-cl * st, -sl * ct, 0.0};
  const TrigLin EYt{0.0, 0.0, st}, NYt{-cl * ct, sl * st, 0.0};    // theta derivatives (EX, NX do not move)
  for (int i = 0; i < 4; ++i)
    for (int m = 0; m < 5; ++m) pc[i][m] = ptc[i][m] = 0.0;
  trig_mul_add(EX, EX, 0.5, pc[0]);
  trig_mul_add(NX, NX, -0.5, pc[0]);
  trig_mul_add(EY, EY, -0.5, pc[0]);
  trig_mul_add(NY, NY, 0.5, pc[0]);
  trig_mul_add(EX, NX, 1.0, pc[1]);
  trig_mul_add(EY, NY, -1.0, pc[1]);
  trig_mul_add(EX, EY, 1.0, pc[2]);
  trig_mul_add(NX, NY, -1.0, pc[2]);
  trig_mul_add(EX, NY, 1.0, pc[3]);
  trig_mul_add(NX, EY, 1.0, pc[3]);
  trig_mul_add(EY, EYt, -1.0, ptc[0]);
  trig_mul_add(NY, NYt, 1.0, ptc[0]);
  trig_mul_add(EYt, NY, -1.0, ptc[1]);
  trig_mul_add(EY, NYt, -1.0, ptc[1]);
  trig_mul_add(EX, EYt, 1.0, ptc[2]);
  trig_mul_add(NX, NYt, -1.0, ptc[2]);
  trig_mul_add(EX, NYt, 1.0, ptc[3]);
  trig_mul_add(NX, EYt, 1.0, ptc[3]);
}

// Pattern maps of one interferometer: F+ = alpha.P, Fx = beta.P.
__host__ __device__ inline void pattern_map(double gamma, double zeta, double c2p, double s2p,
                                            double al[4], double be[4]) {
  const double sz = sin(zeta), s2g = sin(2.0 * gamma), c2g = cos(2.0 * gamma);
  al[0] = sz * s2g * c2p; al[1] = -sz * c2g * c2p; al[2] = sz * s2g * s2p; al[3] = -sz * c2g * s2p;
  be[0] = -sz * s2g * s2p; be[1] = sz * c2g * s2p; be[2] = sz * s2g * c2p; be[3] = -sz * c2g * c2p;
}

// Per (event, site) constants.  A triangle (shape 1) is three 60-degree
// interferometers with bisectors at gamma + 30 deg + k 120 deg; since the
// third arm's response is minus the sum of the other two (closed loop,
// sec. 3.3), the Gram sum over its arms a a^T + b b^T + (a+b)(a+b)^T equals
// (3/2)(a+b)(a+b)^T + (1/2)(a-b)(a-b)^T: two effective interferometers.
// arm_on: bit k set where arm k of the site takes part (the duty factor).
// A triangle with all three arms uses the closure form (two effective
// interferometers with weights 3/2 and 1/2); with some arms off, every arm
// that is on is its own effective interferometer.  A site with no arm on has
// none (its patterns are still set for the strain).
// piM: pi times the event's total mass in seconds (EventC::piM, the only
// event constant a site needs).
__host__ __device__ inline void site_setup(const double* p, const SiteDesc& sd, double piM, SiteC& sc,
                                           uint32_t arm_on = 7u) {
  const double th = p[3], ph = p[4], psi = p[6];
  const double c2p = cos(2.0 * psi), s2p = sin(2.0 * psi);
  sc.cdl = cos(sd.lon - ph);
  sc.sdl = sin(sd.lon - ph);
  const double ct = cos(th), st = sin(th), sl = sin(sd.lat), cl = cos(sd.lat);
  sc.ct = ct; sc.st = st; sc.sl = sl; sc.cl = cl;
  sc.slct = sl * ct;
  sc.clst = cl * st;
  // arrival-time offset -(n . r)/c with n.r/R = sin th cos lat cos H + cos th sin lat
  sc.k1 = -kREarthS * cl * st;
  sc.k0 = -kREarthS * sl * ct;
  sc.k1t = -kREarthS * cl * ct;
  sc.k0t = kREarthS * sl * st;
  sc.lnx_off = -log(piM) - log(sd.f0);
  sc.xp_fac = exp(-4.14 * sc.lnx_off);
  sc.ix_fac = sd.f0 * piM;
  sc.x_fac = 1.0 / sc.ix_fac;
  sc.S0inv = 1.0 / sd.S0;
  sc.xpS0 = sd.S0 * sc.xp_fac;
  sc.m5S0 = -5.0 * sd.S0;
  sc.k111S0 = 111.0 * sd.S0;
  sc.rS0inv = sqrt(sc.S0inv);
  sc.tab_f = sd.tab_f;
  sc.tab_S = sd.tab_S;
  sc.tab_n = sd.tab_n;
  sc.tab_kind = sd.psd_kind;
  sc.pad = 0;
  if (sd.shape == 1) {
    double al[3][4], be[3][4];
    for (int k = 0; k < 3; ++k) {
      pattern_map(sd.gamma + kPi / 6.0 + kTwoPi * k / 3.0, kPi / 3.0, c2p, s2p, al[k], be[k]);
      for (int j = 0; j < 4; ++j) { sc.arm_alpha[k][j] = al[k][j]; sc.arm_beta[k][j] = be[k][j]; }
    }
    sc.n_arm = 3;
    if ((arm_on & 7u) == 7u) {
      for (int j = 0; j < 4; ++j) {
        sc.alpha[0][j] = al[0][j] + al[1][j]; sc.beta[0][j] = be[0][j] + be[1][j];
        sc.alpha[1][j] = al[0][j] - al[1][j]; sc.beta[1][j] = be[0][j] - be[1][j];
      }
      sc.weff[0] = 1.5; sc.weff[1] = 0.5;
      sc.n_eff = 2;
    } else {
      int m = 0;
      for (int k = 0; k < 3; ++k)
        if (arm_on >> k & 1u) {
          for (int j = 0; j < 4; ++j) { sc.alpha[m][j] = al[k][j]; sc.beta[m][j] = be[k][j]; }
          sc.weff[m] = 1.0;
          ++m;
        }
      for (int r = m; r < 2; ++r) {
        for (int j = 0; j < 4; ++j) { sc.alpha[r][j] = 0.0; sc.beta[r][j] = 0.0; }
        sc.weff[r] = 0.0;
      }
      sc.n_eff = m;
    }
  } else {
    pattern_map(sd.gamma, sd.zeta, c2p, s2p, sc.alpha[0], sc.beta[0]);
    for (int j = 0; j < 4; ++j) {
      sc.arm_alpha[0][j] = sc.alpha[0][j]; sc.arm_beta[0][j] = sc.beta[0][j];
      sc.alpha[1][j] = 0.0; sc.beta[1][j] = 0.0;
    }
    sc.weff[0] = 1.0; sc.weff[1] = 0.0;
    sc.n_eff = (arm_on & 1u) ? 1 : 0; sc.n_arm = 1;
  }
  double pc[4][5], ptc[4][5];
  pattern_trig(ct, st, sl, cl, pc, ptc);
  for (int j = 0; j < 2; ++j) {
    const double w = sqrt(sc.weff[j]);
    for (int m = 0; m < 5; ++m) {
      double fp = 0.0, fx = 0.0, fpt = 0.0, fxt = 0.0;
      for (int i = 0; i < 4; ++i) {
        fp = fma(sc.alpha[j][i], pc[i][m], fp);
        fx = fma(sc.beta[j][i], pc[i][m], fx);
        fpt = fma(sc.alpha[j][i], ptc[i][m], fpt);
        fxt = fma(sc.beta[j][i], ptc[i][m], fxt);
      }
      sc.jk[j][0][m] = w * fp;
      sc.jk[j][1][m] = w * fx;
      sc.jk[j][2][m] = w * fpt;
      sc.jk[j][3][m] = w * fxt;
    }
  }
}

__host__ __device__ inline void site_setup(const double* p, const SiteDesc& sd, const EventC& ec, SiteC& sc,
                                           uint32_t arm_on = 7u) {
  site_setup(p, sd, ec.piM, sc, arm_on);
}

// The arm mask of site s for event e from the per-interferometer flags
// active[ifo][ld] (NULL: every arm on); interferometers are numbered site
// by site, three for a triangle, one for an L.
__host__ __device__ inline uint32_t site_arms_on(const uint8_t* active, int64_t ld, int64_t e,
                                                 const NetDesc& net, int s) {
  if (!active) return 7u;
  int ifo0 = 0;
  for (int u = 0; u < s; ++u) ifo0 += net.site[u].shape == 1 ? 3 : 1;
  const int na = net.site[s].shape == 1 ? 3 : 1;
  uint32_t m = 0;
  for (int k = 0; k < na; ++k)
    if (active[(int64_t)(ifo0 + k) * ld + e]) m |= 1u << k;
  return m;
}

// The arms of site s that take part when only interferometer ifo_sel - 1 is
// wanted (ifo_sel = 0: every arm in `arms`).
__host__ __device__ inline uint32_t select_ifo(uint32_t arms, const NetDesc& net, int s, int ifo_sel) {
  if (ifo_sel <= 0) return arms;
  int ifo0 = 0;
  for (int u = 0; u < s; ++u) ifo0 += net.site[u].shape == 1 ? 3 : 1;
  const int k = ifo_sel - 1 - ifo0;
  const int na = net.site[s].shape == 1 ? 3 : 1;
  return (k >= 0 && k < na) ? (arms & (1u << k)) : 0u;
}

// ---------------------------------------------------------- sin and cos
// sin and cos of a moderate angle (|x| < 1e5): Cody-Waite reduction by pi/2
// with a three-part constant, then the Taylor series of sin (to x^17) and
// cos (to x^18) on [-pi/4, pi/4], whose truncation errors (< 1e-19) are far
// below one ulp.  Used for the sidereal angle, which stays within tens of
// radians, instead of a general routine built for arbitrary arguments.
__host__ __device__ inline void sincos_moderate(double x, double* s, double* c) {
  // pi/2 = C1 + C2 + C3 (+1e-37): C1 and C2 are pi/2 and its remainder
  // rounded to 33 significant bits, so k*C1 and k*C2 are exact for |k| < 2^20
  constexpr double kInvPio2 = 0.63661977236758134308;
  constexpr double C1 = 1.5707963267341256e+00;
  constexpr double C2 = 6.077100506303966e-11;
  constexpr double C3 = 2.0222662487959506e-21;
  const double kf = rint(x * kInvPio2);
  double r = fma(-kf, C1, x);
  r = fma(-kf, C2, r);
  r = fma(-kf, C3, r);
  const double r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - ...), cos r = 1 - r^2/2! + r^4/4! - ...
  double ps = -1.0 / 355687428096000.0;          // -1/17!
  ps = fma(ps, r2, 1.0 / 1307674368000.0);       //  1/15!
  ps = fma(ps, r2, -1.0 / 6227020800.0);         // -1/13!
  ps = fma(ps, r2, 1.0 / 39916800.0);            //  1/11!
  ps = fma(ps, r2, -1.0 / 362880.0);             // -1/9!
  ps = fma(ps, r2, 1.0 / 5040.0);                //  1/7!
  ps = fma(ps, r2, -1.0 / 120.0);                // -1/5!
  ps = fma(ps, r2, 1.0 / 6.0);                   //  1/3!
  const double sr = fma(-r * r2, ps, r);
  double pc = 1.0 / 6402373705728000.0;          //  1/18!
  pc = fma(pc, r2, -1.0 / 20922789888000.0);     // -1/16!
  pc = fma(pc, r2, 1.0 / 87178291200.0);         //  1/14!
  pc = fma(pc, r2, -1.0 / 479001600.0);          // -1/12!
  pc = fma(pc, r2, 1.0 / 3628800.0);             //  1/10!
  pc = fma(pc, r2, -1.0 / 40320.0);              // -1/8!
  pc = fma(pc, r2, 1.0 / 720.0);                 //  1/6!
  pc = fma(pc, r2, -1.0 / 24.0);                 // -1/4!
  pc = fma(pc, r2, 0.5);                         //  1/2!
  const double cr = fma(-r2, pc, 1.0);
  const int q = (int)kf & 3;
  const double ss = (q & 1) ? cr : sr;
  const double cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// ------------------------------------------------------ per-point pieces
// Powers of v at one grid point, shared by every PN series of the point.
struct VPow {
  double p1, p2, p3, p4, p5, p6, p7;   // v^1 .. v^7
  double L, Lv;                        // ln v and v ln v
};

__host__ __device__ inline void vpow(double v, double L, VPow& w) {
  w.p1 = v;
  w.p2 = v * v;
  w.p3 = w.p2 * v;
  w.p4 = w.p2 * w.p2;
  w.p5 = w.p4 * v;
  w.p6 = w.p3 * w.p3;
  w.p7 = w.p4 * w.p3;
  w.L = L;
  w.Lv = L * v;
}

// c0 + c1 v + ... + c7 v^7 as a sum of products with the powers, lowest
// order first and c0 last.  Each fused multiply-add keeps the running sum as
// its addend, so per-event coefficients held in scalar registers enter every
// step directly (a Horner recurrence makes the coefficient the addend, which
// costs two register copies per step on this ISA).
__host__ __device__ inline double series7(const double c[8], const VPow& w) {
  double h = c[1] * w.p1;
  h = fma(c[2], w.p2, h);
  h = fma(c[3], w.p3, h);
  h = fma(c[4], w.p4, h);
  h = fma(c[5], w.p5, h);
  h = fma(c[6], w.p6, h);
  h = fma(c[7], w.p7, h);
  return h + c[0];
}

// The same polynomial by Horner's rule, which keeps fewer values live than
// the sum of products (whose coefficient loads the compiler issues all at
// once).  The SNR kernel, which re-reads the coefficients from LDS, uses it;
// the Fisher kernels use the sum, whether their coefficients sit in scalar
// registers or in LDS.
__host__ __device__ inline double horner7(const double c[8], double v) {
  double h = c[7];
  for (int k = 6; k >= 0; --k) h = fma(h, v, c[k]);
  return h;
}
template <bool PSUM>
__host__ __device__ inline double poly7(const double c[8], const VPow& w) {
  return PSUM ? series7(c, w) : horner7(c, w.p1);
}

// A phase series (PhaseSeries) at v: v^-5 (sum c_k v^k) + (l5 + l6 v) ln v
// + t10 v^5 + t12 v^7.
template <bool PSUM = true>
__host__ __device__ inline double eval_phase(const PhaseSeries& s, const VPow& w, double iv5) {
  const double rest = fma(s.l6, w.Lv, fma(s.l5, w.L, fma(s.t12, w.p7, s.t10 * w.p5)));
  return fma(poly7<PSUM>(s.c, w), iv5, rest);
}
// The spin series, whose l6, t10 and t12 are zero by construction.
template <bool PSUM = true>
__host__ __device__ inline double eval_phase_spin(const PhaseSeries& s, const VPow& w, double iv5) {
  return fma(poly7<PSUM>(s.c, w), iv5, s.l5 * w.L);
}
// The deformability series, which only have the tidal terms.
__host__ __device__ inline double eval_phase_tidal(const PhaseSeries& s, const VPow& w) {
  return fma(s.t12, w.p7, s.t10 * w.p5);
}
// A tau*-type series at v: v^-8 (sum c_k v^k) + l6 ln v v^-2.
template <bool PSUM = true>
__host__ __device__ inline double eval_tau(const TauSeries& s, const VPow& w, double iv8, double iv2) {
  return fma(poly7<PSUM>(s.c, w), iv8, s.l6 * (w.L * iv2));
}

// Frequency-point quantities shared by all sites.
struct Point {
  double v, iv, L, f, tf, w4A2;   // tf = 2 pi f; w4A2 = 4 w A^2 (PSD not yet applied)
  double rw;                      // sqrt(w4A2)
  double cth, sth;                // cos, sin of the sidereal angle at t(f)
  double gMc, gEta;               // d(sidereal angle)/dMc, /deta
  double pMc, pEta;               // dPsi_PN/dMc, /deta
  double vpsd;                    // v^-12.42: the PSD's power law, shared by all sites
  double v3, iv3;                 // v^3 and v^-3 (proportional to f and 1/f), shared by all sites
  double ecv;                     // v^-5 (v_ref/v)^{19/3} (eccentric forms, else 0)
};

// v = exp(ln v), 1/v and the PSD's power law v^-12.42 at the points k,
// k + stride, k + 2 stride, ... of a log grid (ln v linear in k): evaluated
// once at the first point, then multiplied by the ratios exp(stride dlnv),
// exp(-stride dlnv), exp(-12.42 stride dlnv) per step.  After m steps each
// value carries a relative error of at most about (2m + 1) u (u = 2^-53) on
// top of that of its first evaluation: 1.4e-14 for the 63 steps of a
// 16384-point work item walked by 256 lanes, far inside the Fisher and SNR
// tolerances, for three multiplications per point instead of two
// exponentials and a reciprocal.
struct GridWalk {
  double val[3];      // v, 1/v, v^-12.42 at the current point
  double ratio[3];
  __host__ __device__ inline void start(const EventC& ec, int32_t k, int32_t stride) {
    const double L = fma((double)k, ec.dlnv, ec.lnv0), D = (double)stride * ec.dlnv;
    val[0] = exp(L);
    val[1] = exp(-L);
    val[2] = exp(-12.42 * L);
    ratio[0] = exp(D);
    ratio[1] = exp(-D);
    ratio[2] = exp(-12.42 * D);
  }
  __host__ __device__ inline void step() {
    val[0] *= ratio[0];
    val[1] *= ratio[1];
    val[2] *= ratio[2];
  }
  // the values at point k evaluated directly again (ratios kept)
  __host__ __device__ inline void anchor(const EventC& ec, int32_t k) {
    const double L = fma((double)k, ec.dlnv, ec.lnv0);
    val[0] = exp(L);
    val[1] = exp(-L);
    val[2] = exp(-12.42 * L);
  }
};

// Number of phase-only Fisher parameters (Phic, chi1z, chi2z, then Lambda1,
// Lambda2 with tides, then e0 with eccentricity) and what it implies.
template <int NPI>
struct PhaseOnly {
  static_assert(NPI >= 3 && NPI <= 6, "3 to 6 phase-only parameters");
  static constexpr bool tidal = NPI >= 5;
  static constexpr bool ecc = (NPI & 1) == 0;
  static constexpr int P = 8 + NPI;
};

// How point_setup forms the PSD's power law v^-12.42 shared by all sites:
// not at all, in FP64, or in FP32 (the mixed form's weight).
enum PsdPow { kPsdNone = 0, kPsdF64 = 1, kPsdF32 = 2 };

// PSUM: the evaluation form of the PN series (see horner7) and of the PSD's
// power law (once per point when true, once per site otherwise).
// EXPL: the point of an explicit grid (ec.fx) rather than of the log grid.
// vrec (log grids only, NULL: evaluate directly): v, 1/v and v^-12.42 at the
// point, carried by the caller from an earlier point (see GridWalk).
template <bool PSUM = true, bool EXPL = false, bool ECC = false>
__host__ __device__ inline void point_setup(const EventC& ec, int32_t k, bool need_derivs, bool rot,
                                            Point& q, int psd = kPsdF64, const double* vrec = nullptr) {
  double L, v, f, wf;               // wf: the trapezoid weight
  double rwe = 0.0;                 // log grid: sqrt(w KA4 / (pi M)) of the point's weight
  if (EXPL) {
    f = ec.fx[k];
    L = (ec.lnpiM + log(f)) / 3.0;
    v = exp(L);
    wf = 0.5 * (ec.fx[k < ec.n - 1 ? k + 1 : k] - ec.fx[k > 0 ? k - 1 : k]);
  } else {
    L = fma((double)k, ec.dlnv, ec.lnv0);
    v = vrec ? vrec[0] : exp(L);
    f = (v * v * v) * ec.inv_piM;
    double w = ec.wint;
    rwe = ec.rwint;
    if (k == 0) {
      w = ec.wfirst;
      rwe = ec.rwfirst;
    }
    if (k == ec.n - 1) {
      w = ec.wlast;
      rwe = ec.rwlast;
    }
    wf = w * f;
  }
  const double iv = (!EXPL && vrec) ? vrec[1] : recip(v);
  const double iv2 = iv * iv, iv4 = iv2 * iv2, iv5 = iv4 * iv, iv7 = iv5 * iv2, iv8 = iv4 * iv4;
  q.v = v; q.iv = iv; q.L = L; q.f = f;
  q.v3 = v * v * v;
  q.iv3 = iv2 * iv;
  q.tf = kTwoPi * f;
  q.w4A2 = wf * ec.KA4 * iv7;
  q.rw = EXPL ? sqrt(q.w4A2) : rwe * iv2;
  q.vpsd = 0.0;
  if (!EXPL && vrec && psd != kPsdNone) {
    q.vpsd = vrec[2];
  } else if (PSUM && psd == kPsdF64) {
    q.vpsd = exp(-12.42 * L);
  } else if (psd == kPsdF32) {   // 2^y with the integer part of y split off exactly
    const double y = (-12.42 / kLn2) * L, ny = rint(y);
    q.vpsd = (double)ldexpf(exp2f((float)(y - ny)), (int)ny);
  }
  VPow pw;
  vpow(v, L, pw);
  const double th = rot ? ec.thc + eval_tau<PSUM>(ec.ts[kTsTheta], pw, iv8, iv2) : ec.thc;
  sincos_moderate(th, &q.sth, &q.cth);
  if (need_derivs) {
    q.gMc = rot ? eval_tau<PSUM>(ec.ts[kTsMc], pw, iv8, iv2) : 0.0;
    q.gEta = rot ? eval_tau<PSUM>(ec.ts[kTsEta], pw, iv8, iv2) : 0.0;
    q.pMc = eval_phase<PSUM>(ec.ps[kPsMc], pw, iv5);
    q.pEta = eval_phase<PSUM>(ec.ps[kPsEta], pw, iv5);
  }
  q.ecv = 0.0;
  if (ECC) {
    q.ecv = iv5 * exp((19.0 / 3.0) * (ec.ecc_lnvr - L));
    if (need_derivs) q.pMc = fma(ec.ecc_mc, q.ecv, q.pMc);
  }
}

// The phase-only derivative coefficients of a point: c = (-1, dPsi/dchi1,
// dPsi/dchi2[, dPsi/dLambda1, dPsi/dLambda2][, dPsi/de0]).
template <int NPI, bool PSUM = true>
__host__ __device__ inline void phase_only_coefficients(const EventC& ec, const Point& q, double* c) {
  using PO = PhaseOnly<NPI>;
  const double iv = q.iv, iv2 = iv * iv, iv5 = iv2 * iv2 * iv;
  VPow pw;
  vpow(q.v, q.L, pw);
  c[0] = -1.0;
  if (PSUM) {      // the spin and deformability series' structural zeros skipped
    c[1] = eval_phase_spin<true>(ec.ps[kPsChi1], pw, iv5);
    c[2] = eval_phase_spin<true>(ec.ps[kPsChi2], pw, iv5);
    if (PO::tidal) {
      c[3] = eval_phase_tidal(ec.ps[kPsL1], pw);
      c[4] = eval_phase_tidal(ec.ps[kPsL2], pw);
    }
  } else {         // the general form (fewer live values)
    c[1] = eval_phase<false>(ec.ps[kPsChi1], pw, iv5);
    c[2] = eval_phase<false>(ec.ps[kPsChi2], pw, iv5);
    if (PO::tidal) {
      c[3] = eval_phase<false>(ec.ps[kPsL1], pw, iv5);
      c[4] = eval_phase<false>(ec.ps[kPsL2], pw, iv5);
    }
  }
  if (PO::ecc) c[NPI - 1] = ec.ecc_e0 * q.ecv;
}

// Site-level quantities at one frequency: the P vectors and their hour-angle
// and theta derivatives, the delay derivatives and the noise weight.
struct SitePoint {
  double P[4], PH[4], Pt[4];
  double dH, dT;      // dDelta/dH, dDelta/dtheta
  double om;          // 4 w A^2 / S_n(f)
};

template <bool PSUM = true>
__host__ __device__ inline double psd_weight_of(double xp_fac, double lnx_off, double ix_fac,
                                                double x_fac, double S0inv, const Point& q) {
  // S_n = S0 [x^-4.14 - 5 x^-2 + 111 (1 - x^2 + x^4/2)/(1 + x^2/2)], x = f/f0;
  // x^-4.14 = xp_fac v^-12.42 with the power of v evaluated once per point
  // (PSUM), or exp(-4.14 ln x) here
  const double xp = PSUM ? xp_fac * q.vpsd : exp(-4.14 * fma(3.0, q.L, lnx_off));
  const double ix = ix_fac * q.iv3;                // f0/f
  const double x = x_fac * q.v3;                   // f/f0
  const double ix2 = ix * ix;
  const double x2 = x * x;
  const double num = fma(0.5 * x2, x2, 1.0 - x2);
  const double den = fma(0.5, x2, 1.0);
  // shape = [(x^-4.14 - 5 x^-2) den + 111 num] / den
  const double top = fma(fma(-5.0, ix2, xp), den, 111.0 * num);
  return q.w4A2 * S0inv * den * recip(top);
}

// The weight with a sampled noise curve (sec. 3.1, a PSD or ASD file): the
// PSD between two samples on the straight line through them (an ASD squared
// at the samples first), scaled by S0; no weight outside the sampled range,
// whose end samples cover frequencies within a relative 1e-12 of them (so a
// grid starting on a sampled frequency keeps its first point whatever the
// rounding of f).  The interval is found by bisection over the samples.
__host__ __device__ inline double table_weight(const double* __restrict__ tf, const double* __restrict__ tS,
                                               int64_t n, int32_t kind, double S0inv, double w4A2, double f) {
  constexpr double eps = 1e-12;
  if (!(f >= tf[0] * (1.0 - eps)) || !(f <= tf[n - 1] * (1.0 + eps))) return 0.0;
  int64_t lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (tf[mid] <= f) lo = mid;
    else hi = mid;
  }
  double s0 = tS[lo], s1 = tS[hi];
  if (kind == 2) {
    s0 *= s0;
    s1 *= s1;
  }
  const double t = fmin(fmax((f - tf[lo]) / (tf[hi] - tf[lo]), 0.0), 1.0);
  return w4A2 * S0inv / fma(t, s1 - s0, s0);
}

// TAB = false: instantiations for networks without sampled curves, which
// leave the check out of the per-point code.
template <bool PSUM = true, bool TAB = true>
__host__ __device__ inline void psd_weight(const SiteC& sc, const Point& q, double& om) {
  if (TAB && sc.tab_kind) om = table_weight(sc.tab_f, sc.tab_S, sc.tab_n, sc.tab_kind, sc.S0inv, q.w4A2, q.f);
  else om = psd_weight_of<PSUM>(sc.xp_fac, sc.lnx_off, sc.ix_fac, sc.x_fac, sc.S0inv, q);
}

// The same weight with the PSD shape evaluated in FP32 (mixed form).  The
// weight is a positive factor per grid point, so a relative error e in it
// keeps the Fisher matrix between (1 - e) Gamma and (1 + e) Gamma in the
// positive-semidefinite order: SNR^2 moves by at most e and every sigma_i by
// at most about e/2, whatever the condition number.  Errors in the
// derivative vectors or in the sums have no such bound, which is why they
// stay FP64.  x^-4.14 = xp_fac v^-12.42, the power of v taken once per point
// as 2^y with y = -12.42 log2 v formed in FP64 and its integer part split
// off exactly (point_setup, kPsdF32), so the FP32 exponential sees
// |r| <= 1/2; x^2 and x^-2 are FP64 products rounded once; the quotient uses
// the FP32 reciprocal.
template <bool TAB = true>
__host__ __device__ inline void psd_weight_f32(const SiteC& sc, const Point& q, double& om) {
  if (TAB && sc.tab_kind) {   // a sampled curve: the FP64 weight
    om = table_weight(sc.tab_f, sc.tab_S, sc.tab_n, sc.tab_kind, sc.S0inv, q.w4A2, q.f);
    return;
  }
  const float xp = (float)(sc.xp_fac * q.vpsd);
  const double x = sc.x_fac * q.v3, ix = sc.ix_fac * q.iv3;
  const float x2 = (float)(x * x), ix2 = (float)(ix * ix);
  const float num = fmaf(0.5f * x2, x2, 1.0f - x2);
  const float den = fmaf(0.5f, x2, 1.0f);
  const float top = fmaf(fmaf(-5.0f, ix2, xp), den, 111.0f * num);
  om = q.w4A2 * sc.S0inv * (double)(den * recipf(top));
}

// The square root of the weight, r = sqrt(4 w A^2 / S_n(f)), which the
// Fisher kernels fold into the pattern values: every Fisher entry is a sum of
// w Re(D_a D_b^*), bilinear in the derivative vectors, and those are linear
// in the pattern values, so the weighted sums follow from r D with no
// per-entry weight product.  With S_n = S0 top / den (psd_weight_of),
// r = sqrt(4 w A^2) den / sqrt(den S0 top); S0 top is formed from the site's
// S0-scaled coefficients, so 1/S0 costs nothing per point.  A sampled curve,
// and the per-site evaluation of the power law (PSUM = false), take the root
// of the full weight.
template <bool PSUM = true, bool TAB = true>
__host__ __device__ inline double psd_root_weight(const SiteC& sc, const Point& q) {
  if ((TAB && sc.tab_kind) || !PSUM) {
    double om;
    psd_weight<PSUM, TAB>(sc, q, om);
    return sqrt(om);
  }
  const double ix = sc.ix_fac * q.iv3;             // f0/f
  const double x = sc.x_fac * q.v3;                // f/f0
  const double ix2 = ix * ix;
  const double x2 = x * x;
  const double num = fma(0.5 * x2, x2, 1.0 - x2);
  const double den = fma(0.5, x2, 1.0);
  const double topS = fma(fma(sc.m5S0, ix2, sc.xpS0 * q.vpsd), den, sc.k111S0 * num);
  return (q.rw * den) * rsqrt_d(den * topS);
}

// The same root in the mixed form: the shape as in psd_weight_f32,
// sqrt(den / top) in FP32 (den/top = S0/S_n stays within FP32's range), so a
// relative error e in r is one of about 2e in the weight, the positive factor
// whose error psd_weight_f32 bounds.  Measured on sampled events of the BNS
// catalogue: Fisher within 4.2e-8 of sqrt(Gamma_aa Gamma_bb), SNR within 1.9e-8.
template <bool TAB = true>
__host__ __device__ inline double psd_root_weight_f32(const SiteC& sc, const Point& q) {
  if (TAB && sc.tab_kind)
    return sqrt(table_weight(sc.tab_f, sc.tab_S, sc.tab_n, sc.tab_kind, sc.S0inv, q.w4A2, q.f));
  const float xp = (float)(sc.xp_fac * q.vpsd);
  const double x = sc.x_fac * q.v3, ix = sc.ix_fac * q.iv3;
  const float x2 = (float)(x * x), ix2 = (float)(ix * ix);
  const float num = fmaf(0.5f * x2, x2, 1.0f - x2);
  const float den = fmaf(0.5f, x2, 1.0f);
  const float top = fmaf(fmaf(-5.0f, ix2, xp), den, 111.0f * num);
  return (q.rw * sc.rS0inv) * (double)sqrtf_hw(den * recipf(top));
}

template <bool MIXED = false, bool PSUM = true, bool TAB = true>
__host__ __device__ inline void site_point(const SiteC& sc, const Point& q, bool need_derivs,
                                           SitePoint& sp) {
  const double cH = q.cth * sc.cdl - q.sth * sc.sdl;
  const double sH = q.sth * sc.cdl + q.cth * sc.sdl;
  const double EX = cH, EY = -sc.ct * sH, NX = -sc.sl * sH, NY = -(sc.slct * cH + sc.clst);
  sp.P[0] = 0.5 * (EX * EX - NX * NX - EY * EY + NY * NY);
  sp.P[1] = EX * NX - EY * NY;
  sp.P[2] = EX * EY - NX * NY;
  sp.P[3] = EX * NY + NX * EY;
  if (MIXED) psd_weight_f32<TAB>(sc, q, sp.om);
  else psd_weight<PSUM, TAB>(sc, q, sp.om);
  if (!need_derivs) return;
  const double EXh = -sH, EYh = -sc.ct * cH, NXh = -sc.sl * cH, NYh = sc.slct * sH;
  sp.PH[0] = EX * EXh - NX * NXh - EY * EYh + NY * NYh;
  sp.PH[1] = EXh * NX + EX * NXh - EYh * NY - EY * NYh;
  sp.PH[2] = EXh * EY + EX * EYh - NXh * NY - NX * NYh;
  sp.PH[3] = EXh * NY + EX * NYh + NXh * EY + NX * EYh;
  const double EYt = sc.st * sH, NYt = sc.sl * sc.st * cH - sc.cl * sc.ct;
  sp.Pt[0] = -EY * EYt + NY * NYt;
  sp.Pt[1] = -(EYt * NY + EY * NYt);
  sp.Pt[2] = EX * EYt - NX * NYt;
  sp.Pt[3] = EX * NYt + NX * EYt;
  sp.dH = -sc.k1 * sH;
  sp.dT = fma(sc.k1t, cH, sc.k0t);
}

// Site-level quantities of the Fisher kernels at one frequency for the
// trigonometric form of the patterns (SiteC::jk): cos H, sin H, cos 2H,
// sin 2H and the factors 2 cos 2H, -2 sin 2H of the H derivatives; the
// arrival-time derivatives and the noise weight.
struct SiteTrig {
  double cH, sH, c2H, s2H, p2c, m2s;
  double dH, dT;      // dDelta/dH, dDelta/dtheta
  double om;          // 4 w A^2 / S_n(f)
};

template <bool MIXED = false, bool PSUM = true, bool TAB = true>
__host__ __device__ inline void site_trig(const SiteC& sc, const Point& q, SiteTrig& sp) {
  const double cH = q.cth * sc.cdl - q.sth * sc.sdl;
  const double sH = q.sth * sc.cdl + q.cth * sc.sdl;
  sp.cH = cH;
  sp.sH = sH;
  sp.c2H = fma(cH, cH, -sH * sH);
  sp.s2H = 2.0 * (sH * cH);
  sp.p2c = 2.0 * sp.c2H;
  sp.m2s = -2.0 * sp.s2H;
  if (MIXED) psd_weight_f32<TAB>(sc, q, sp.om);
  else psd_weight<PSUM, TAB>(sc, q, sp.om);
  sp.dH = -sc.k1 * sH;
  sp.dT = fma(sc.k1t, cH, sc.k0t);
}

// The Fisher kernels' site quantities: the patterns' trigonometric basis
// scaled by the root weight r (psd_root_weight), so that SiteC::jk's
// polynomials give r F+, r Fx and their derivatives directly; cos H and
// sin H themselves for the arrival-time derivatives.
struct SiteTrigR {
  double cH, sH;
  double r, rc, rs, rc2, rs2;   // r (1, cos H, sin H, cos 2H, sin 2H)
  double p2c, m2s;              // r (2 cos 2H, -2 sin 2H)
  double dH, dT;                // dDelta/dH, dDelta/dtheta
};

template <bool MIXED = false, bool PSUM = true, bool TAB = true>
__host__ __device__ inline void site_trig_root(const SiteC& sc, const Point& q, SiteTrigR& sp) {
  const double cH = q.cth * sc.cdl - q.sth * sc.sdl;
  const double sH = q.sth * sc.cdl + q.cth * sc.sdl;
  sp.cH = cH;
  sp.sH = sH;
  const double r = MIXED ? psd_root_weight_f32<TAB>(sc, q) : psd_root_weight<PSUM, TAB>(sc, q);
  sp.r = r;
  sp.rc = r * cH;
  sp.rs = r * sH;
  sp.rc2 = fma(sp.rc, cH, -sp.rs * sH);
  sp.rs2 = 2.0 * (sp.rs * cH);
  sp.p2c = 2.0 * sp.rc2;
  sp.m2s = -2.0 * sp.rs2;
  sp.dH = -sc.k1 * sH;
  sp.dT = fma(sc.k1t, cH, sc.k0t);
}

// r times a trigonometric polynomial of SiteC::jk, and r times its H
// derivative (the constant term last, as in trig_val).
__host__ __device__ inline double trig_val_r(const double c[5], const SiteTrigR& sp) {
  return fma(c[0], sp.r, fma(c[4], sp.rs2, fma(c[3], sp.rc2, fma(c[2], sp.rs, c[1] * sp.rc))));
}
__host__ __device__ inline double trig_dH_r(const double c[5], const SiteTrigR& sp) {
  return fma(c[4], sp.p2c, fma(c[3], sp.m2s, fma(c[2], sp.rc, -c[1] * sp.rs)));
}

// A trigonometric polynomial of SiteC::jk at the point, and its H derivative.
// The constant term is added last: the coefficients sit in scalar registers,
// and as the first addend it would need copying into vector registers.
__host__ __device__ inline double trig_val(const double c[5], const SiteTrig& sp) {
  return fma(c[4], sp.s2H, fma(c[3], sp.c2H, fma(c[2], sp.sH, c[1] * sp.cH))) + c[0];
}
__host__ __device__ inline double trig_dH(const double c[5], const SiteTrig& sp) {
  return fma(c[4], sp.p2c, fma(c[3], sp.m2s, fma(c[2], sp.cH, -c[1] * sp.sH)));
}

__host__ __device__ inline double dot4(const double a[4], const double b[4]) {
  return fma(a[0], b[0], fma(a[1], b[1], fma(a[2], b[2], a[3] * b[3])));
}

// The event's amplitude factors that enter the derivative vectors.
struct AmpFactors {
  double cplus, ccross, dcp, dcx, dlnA, idL;
};

__host__ __device__ inline AmpFactors amp_factors(const EventC& ec) {
  return AmpFactors{ec.cplus, ec.ccross, ec.dcplus, ec.dcross, ec.dlnA_dMc, ec.inv_dL};
}

// A site's derivatives of the phase at one point (the delay's share
// included): with respect to Mc, eta, theta, phi and tc [s].
struct SitePhase {
  double mc, eta, t, p, tc;
};

__host__ __device__ inline SitePhase site_phase(const Point& q, double dH, double dT) {
  return SitePhase{fma(q.tf * dH, q.gMc, q.pMc), fma(q.tf * dH, q.gEta, q.pEta), q.tf * dT,
                   -q.tf * dH, q.tf * fma(kOmegaE, dH, 1.0)};
}
__host__ __device__ inline SitePhase site_phase(const Point& q, const SitePoint& sp) {
  return site_phase(q, sp.dH, sp.dT);
}

// Phase-free derivative vector of one interferometer at one point,
// D_b = dQ_b + Q dlnA_b + i Q dPsi_b for b = (Mc, eta, dL, theta, phi, iota,
// psi, tc), from its pattern values F = (alpha.P, beta.P) and their hour-angle
// (H) and theta (t) derivatives; Q = c+ F+ + i cx Fx.  The strain derivative
// is A exp(i Psi) D_b, and i Q c(f) for the phase-only parameters.
__host__ __device__ inline void derivative_vector(const AmpFactors& am, const Point& q, const SitePhase& ph,
                                                  double Fp, double Fx, double FpH, double FxH,
                                                  double Fpt, double Fxt, double* Dr, double* Di) {
  const double Qr = am.cplus * Fp, Qi = am.ccross * Fx;
  const double QHr = am.cplus * FpH, QHi = am.ccross * FxH;
  const double Qtr = am.cplus * Fpt, Qti = am.ccross * Fxt;
  // D = dQ + Q dlnA + i Q dPsi, with i Q x = (-Qi x, Qr x)
  Dr[0] = fma(Qr, am.dlnA, fma(QHr, q.gMc, -Qi * ph.mc));     // Mc
  Di[0] = fma(Qi, am.dlnA, fma(QHi, q.gMc, Qr * ph.mc));
  Dr[1] = fma(QHr, q.gEta, -Qi * ph.eta);                     // eta
  Di[1] = fma(QHi, q.gEta, Qr * ph.eta);
  Dr[2] = -Qr * am.idL;                                       // dL
  Di[2] = -Qi * am.idL;
  Dr[3] = fma(-Qi, ph.t, Qtr);                                // theta
  Di[3] = fma(Qr, ph.t, Qti);
  Dr[4] = fma(-Qi, ph.p, -QHr);                               // phi (H = ... - phi)
  Di[4] = fma(Qr, ph.p, -QHi);
  Dr[5] = am.dcp * Fp;                                        // iota
  Di[5] = am.dcx * Fx;
  Dr[6] = 2.0 * am.cplus * Fx;                                // psi: dF+ = 2Fx, dFx = -2F+
  Di[6] = -2.0 * am.ccross * Fp;
  Dr[7] = fma(kOmegaE, QHr, -Qi * ph.tc);                     // tc [s]
  Di[7] = fma(kOmegaE, QHi, Qr * ph.tc);
}

// ------------------------------------------------ one frequency point
// The rows of dL, iota and psi are fixed per-event combinations of the
// pattern values (F+, Fx) of each interferometer:
//   D_dL = -Q/dL,  D_iota = (dc+ F+, dcx Fx),  D_psi = (2 c+ Fx, -2 cx F+),
// with Q = (c+ F+, cx Fx) and (re, im) pairs.  So every Fisher entry in
// those rows is a combination of the moments
//   T_b = sum w (F+ Dr_b, F+ Di_b, Fx Dr_b, Fx Di_b)   for the other rows b
//   S   = sum w (F+^2, F+ Fx, Fx^2),
// and only the 5x5 block of (Mc, eta, theta, phi, tc) needs a rank-2 update
// per interferometer.  The accumulator G[kGramAcc] holds that block's upper
// triangle (15, row-major), then T (4 per row, in the order above), then S;
// gram_finish turns it into the 8x8 block.
constexpr int kGramAcc = 15 + 20 + 3;
constexpr int kGramRows[5] = {0, 1, 3, 4, 7};   // Mc, eta, theta, phi, tc

// Adds the contribution of grid point k of an event to G[kGramAcc] (above)
// and returns the point's phase-only quantities:
//   U[8]   U_b = sum_i w_i Re(i Q_i D_b,i^*)
//   W      sum_i w_i |Q_i|^2 (the SNR^2 density)
//   c[NPI] (-1, dPsi/dchi1, dPsi/dchi2[, dPsi/dLambda1, dPsi/dLambda2][, dPsi/de0]).
// The phase-only derivative vectors are i Q c(f) with the same real c(f) at
// every interferometer, so the blocks they span are
//   Gamma_{b, 8+i} += U_b c_i,   Gamma_{8+i, 8+j} += W c_i c_j,
// which the caller accumulates (see add_phase_blocks).  U and W of the rows
// dL, iota, psi follow from the point's moments S as well: U_dL = 0
// exactly, U_iota = (c+ dcx - cx dc+) S_+x, U_psi = -2 c+ cx (S_++ + S_xx),
// W = c+^2 S_++ + cx^2 S_xx.
template <int NPI, bool ROT, bool MIXED = false, bool PSUM = true, bool EXPL = false, bool TAB = true>
__host__ __device__ inline void accumulate_point(const EventC& ec, const SiteC* sc, int n_site,
                                                 int32_t k, double* G, double* U, double& W,
                                                 double* cph, const double* vrec = nullptr) {
  const AmpFactors am = amp_factors(ec);
  Point q;
  point_setup<PSUM, EXPL, PhaseOnly<NPI>::ecc>(ec, k, true, ROT, q, MIXED ? kPsdF32 : kPsdF64, vrec);
  double UR[5], spp = 0.0, spx = 0.0, sxx = 0.0;
#pragma unroll
  for (int b = 0; b < 5; ++b) UR[b] = 0.0;
  for (int s = 0; s < n_site; ++s) {
    const SiteC& st = sc[s];
    SiteTrigR sp;
    site_trig_root<MIXED, PSUM, TAB>(st, q, sp);
    const SitePhase ph = site_phase(q, sp.dH, sp.dT);
    // at most two effective interferometers per site; the count is the same
    // for every lane, so the second pass is skipped as a whole where unused.
    // The patterns are trigonometric polynomials in H whose coefficients
    // carry sqrt(weff), and the basis carries the root weight r, so Fp, Fx,
    // the derivative vectors and Q below are r times their unweighted values
    // and every product of two of them is weighted by w = weff r^2.
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j >= st.n_eff) break;
      const double(*c)[5] = st.jk[j];
      const double Fp = trig_val_r(c[0], sp), Fx = trig_val_r(c[1], sp);
      double Dr[8], Di[8];
      derivative_vector(am, q, ph, Fp, Fx, trig_dH_r(c[0], sp), trig_dH_r(c[1], sp), trig_val_r(c[2], sp),
                        trig_val_r(c[3], sp), Dr, Di);
      const double Qr = am.cplus * Fp, Qi = am.ccross * Fx;
      int g = 0;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const int r = kGramRows[a];
        const double dr = Dr[r], di = Di[r];
#pragma unroll
        for (int b = a; b < 5; ++b) {
          const int c = kGramRows[b];
          G[g] = fma(dr, Dr[c], fma(di, Di[c], G[g]));
          ++g;
        }
        G[15 + 4 * a + 0] = fma(Fp, dr, G[15 + 4 * a + 0]);
        G[15 + 4 * a + 1] = fma(Fp, di, G[15 + 4 * a + 1]);
        G[15 + 4 * a + 2] = fma(Fx, dr, G[15 + 4 * a + 2]);
        G[15 + 4 * a + 3] = fma(Fx, di, G[15 + 4 * a + 3]);
        // w Re(i Q D_r^*) = (r Qr)(r Di_r) - (r Qi)(r Dr_r)
        UR[a] = fma(Qr, di, fma(-Qi, dr, UR[a]));
      }
      spp = fma(Fp, Fp, spp);
      spx = fma(Fp, Fx, spx);
      sxx = fma(Fx, Fx, sxx);
    }
  }
  G[35] += spp;
  G[36] += spx;
  G[37] += sxx;
#pragma unroll
  for (int a = 0; a < 5; ++a) U[kGramRows[a]] = UR[a];
  U[2] = 0.0;
  U[5] = ec.u_iota * spx;
  U[6] = ec.u_psi * (spp + sxx);
  W = fma(ec.cp2, spp, ec.cx2 * sxx);
  phase_only_coefficients<NPI, PSUM>(ec, q, cph);
}

// The 8x8 upper-triangle block of (Mc, eta, dL, theta, phi, iota, psi, tc)
// (row-major, 36 values) from the accumulator of accumulate_point.
__host__ __device__ inline void gram_finish(const EventC& ec, const double* G, double* F) {
  const AmpFactors am = amp_factors(ec);
  auto at = [](int r, int c) { return r <= c ? 8 * r - (r * (r - 1)) / 2 + (c - r)
                                             : 8 * c - (c * (c - 1)) / 2 + (r - c); };
  int g = 0;
  for (int a = 0; a < 5; ++a)
    for (int b = a; b < 5; ++b) F[at(kGramRows[a], kGramRows[b])] = G[g++];
  for (int a = 0; a < 5; ++a) {
    const int r = kGramRows[a];
    const double tpr = G[15 + 4 * a], tpi = G[16 + 4 * a], txr = G[17 + 4 * a], txi = G[18 + 4 * a];
    F[at(r, 2)] = -am.idL * fma(am.cplus, tpr, am.ccross * txi);
    F[at(r, 5)] = fma(am.dcp, tpr, am.dcx * txi);
    F[at(r, 6)] = 2.0 * fma(am.cplus, txr, -am.ccross * tpi);
  }
  const double spp = G[35], spx = G[36], sxx = G[37];
  const double ci = am.ccross, si2 = (1.0 - ci) * (1.0 + ci);   // c+^2 - cx^2 = sin^4(iota)/4
  F[at(2, 2)] = am.idL * am.idL * fma(am.cplus * am.cplus, spp, ci * ci * sxx);
  F[at(2, 5)] = -am.idL * fma(am.cplus * am.dcp, spp, ci * am.dcx * sxx);
  F[at(2, 6)] = -am.idL * 0.5 * si2 * si2 * spx;
  F[at(5, 5)] = fma(am.dcp * am.dcp, spp, am.dcx * am.dcx * sxx);
  F[at(5, 6)] = 2.0 * fma(am.cplus, am.dcp, -ci * am.dcx) * spx;
  F[at(6, 6)] = 4.0 * fma(am.cplus * am.cplus, sxx, ci * ci * spp);
}

// Plain accumulation of the phase-only blocks of one point into
// xy[(b*NPI + i)*xs] (b < 8) and then the upper triangle of W c_i c_j.
__host__ __device__ inline void add_phase_blocks(int NPI, const double* U, double W, const double* cph,
                                                 double* xy, int xs) {
  for (int b = 0; b < 8; ++b)
    for (int i = 0; i < NPI; ++i) xy[(b * NPI + i) * xs] = fma(U[b], cph[i], xy[(b * NPI + i) * xs]);
  int y = 8 * NPI;
  for (int i = 0; i < NPI; ++i) {
    const double wc = W * cph[i];
    for (int j = i; j < NPI; ++j) {
      xy[y * xs] = fma(wc, cph[j], xy[y * xs]);
      ++y;
    }
  }
}

// Position (r, c) in the P x P Fisher matrix of accumulator slot t, with
// slots ordered as: 36 entries of the 8x8 upper block (row-major), then the
// 8 x NPI block, then the NPI x NPI upper block.
__host__ __device__ inline void slot_position(int t, int NPI, int& r, int& c) {
  if (t < 36) {
    int i = t;
    r = 0;
    while (i >= 8 - r) { i -= 8 - r; ++r; }
    c = r + i;
  } else if (t < 36 + 8 * NPI) {
    const int i = t - 36;
    r = i / NPI;
    c = 8 + i % NPI;
  } else {
    int i = t - 36 - 8 * NPI;
    r = 0;
    while (i >= NPI - r) { i -= NPI - r; ++r; }
    c = 8 + r + i;
    r = 8 + r;
  }
}

}  // namespace gwf

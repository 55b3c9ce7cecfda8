// gwf_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow FP64 CPU reference ("the oracle") for the Fisher/SNR path of
// the GWFAST method (arXiv:2207.06910).  Only the test-suite, the smoke
// check and the CPU-baseline leg of the benchmark may load it; the product
// path never does.  It shares no source with the GPU library.
//
// What it computes, literally as defined:
//   * the TaylorF2 restricted-PN strain of a compact binary (sec. 2.2), with
//     aligned spins and the tidal terms built from the combinations of
//     eq. (LamTdelLam_def);
//   * its projection onto each interferometer with antenna patterns written
//     as a contraction of the 3D detector tensor with the polarisation
//     tensors, evaluated at the time t(f) = tc - tau*(f) so that the Earth's
//     rotation enters both the patterns and the arrival-time (Doppler) phase
//     (sec. 3, footnote on Earth motion; tau* at 3.5PN as cited in sec. 2.2);
//   * SNR_i^2 = 4 int |h_i|^2 / S_n,i df and the network sum (sec. 3.2);
//   * Gamma_ij = 4 Re int d_i h d_j h^* / S_n df summed over interferometers
//     (sec. 3.2), with all derivatives taken by forward-mode dual numbers,
//     the same mathematics as the automatic differentiation the paper uses
//     (sec. 3.3);
//   * quadrature: the trapezoid rule on the log-spaced grid the paper builds
//     with geomspace (sec. 2.2), summed with Neumaier compensation.
//
// Where the paper is silent (PN coefficients, constants, sign and frame
// conventions) each block below names the source or the convention it
// follows.  The scalar type is a template parameter so that the
// same code runs on double, on dual numbers (derivatives), on nested dual
// numbers (gradients of Fisher figures of merit w.r.t. detector parameters)
// and on std::complex<double> (complex-step derivative checks).

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------- constants
// The paper fixes none of these numerically; IAU 2015 nominal values.
constexpr double PI = 3.14159265358979323846;
const double C_SI = 299792458.0;                       // m/s
const double GM_SUN = 1.3271244e20;                    // m^3/s^2
const double T_SUN = GM_SUN / (C_SI * C_SI * C_SI);    // G Msun / c^3 [s]
const double AU_M = 149597870700.0;                    // m
const double PC_M = AU_M * 648000.0 / PI;              // m
const double GPC_S = 1e9 * PC_M / C_SI;                // 1 Gpc / c [s]
const double SIDEREAL_DAY = 86164.0905;                // s
const double OMEGA_E = 2.0 * PI / SIDEREAL_DAY;        // rad/s
const double R_EARTH = 6.371e6;                        // m (spherical Earth)
const double EULER_GAMMA = 0.5772156649015329;

enum : int { FLAG_EARTH_ROT = 1, FLAG_TIDAL = 2, FLAG_ECC = 8 };
enum : int { NPAR = 13 };

// ------------------------------------------------------------ dual numbers
// Forward-mode automatic differentiation: value plus N partials.
template <class T, int N>
struct Dual {
  T v;
  T d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = T(0.0); }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = T(0.0); }
  static Dual lift(const T& x) { Dual r; r.v = x; return r; }
};

template <class X> struct is_dual { static constexpr bool value = false; };
template <class T, int N> struct is_dual<Dual<T, N>> { static constexpr bool value = true; };

template <class T, int N>
Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = -a.v;
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <class T, int N>
Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
template <class T, int N> Dual<T, N> operator+(const Dual<T, N>& a, double b) { Dual<T, N> r = a; r.v = r.v + b; return r; }
template <class T, int N> Dual<T, N> operator+(double b, const Dual<T, N>& a) { return a + b; }
template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a, double b) { Dual<T, N> r = a; r.v = r.v - b; return r; }
template <class T, int N> Dual<T, N> operator-(double b, const Dual<T, N>& a) { return (-a) + b; }
template <class T, int N> Dual<T, N> operator*(const Dual<T, N>& a, double b) {
  Dual<T, N> r; r.v = a.v * b;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <class T, int N> Dual<T, N> operator*(double b, const Dual<T, N>& a) { return a * b; }
template <class T, int N> Dual<T, N> operator/(const Dual<T, N>& a, double b) { return a * (1.0 / b); }
template <class T, int N> Dual<T, N> operator/(double b, const Dual<T, N>& a) { return Dual<T, N>(b) / a; }

// Chain rule for a scalar function with value fv and derivative dfv at a.v.
template <class T, int N>
Dual<T, N> chain(const Dual<T, N>& a, const T& fv, const T& dfv) {
  Dual<T, N> r; r.v = fv;
  for (int i = 0; i < N; ++i) r.d[i] = dfv * a.d[i];
  return r;
}
template <class T, int N> Dual<T, N> sin(const Dual<T, N>& a) { using std::sin; using std::cos; return chain(a, sin(a.v), cos(a.v)); }
template <class T, int N> Dual<T, N> cos(const Dual<T, N>& a) { using std::sin; using std::cos; return chain(a, cos(a.v), -sin(a.v)); }
template <class T, int N> Dual<T, N> exp(const Dual<T, N>& a) { using std::exp; T e = exp(a.v); return chain(a, e, e); }
template <class T, int N> Dual<T, N> log(const Dual<T, N>& a) { using std::log; return chain(a, log(a.v), T(1.0) / a.v); }
template <class T, int N> Dual<T, N> sqrt(const Dual<T, N>& a) { using std::sqrt; T s = sqrt(a.v); return chain(a, s, T(0.5) / s); }
template <class T, int N> Dual<T, N> pow(const Dual<T, N>& a, double p) {
  using std::pow;
  return chain(a, pow(a.v, p), T(p) * pow(a.v, p - 1.0));
}

// Promote a detector-parameter value of type T to the working scalar S.
template <class S, class T> struct Lift { static S go(const T& x) { return S(x); } };
template <class T, int N> struct Lift<Dual<T, N>, T> { static Dual<T, N> go(const T& x) { return Dual<T, N>::lift(x); } };
template <class S, class T> S lift(const T& x) { return Lift<S, T>::go(x); }

// Real value of any scalar type used here.
inline double val(double x) { return x; }
inline double val(const std::complex<double>& x) { return x.real(); }
template <class T, int N> double val(const Dual<T, N>& x) { return val(x.v); }

// ------------------------------------------------------------ summation
// Neumaier's compensated summation.
struct NeumaierSum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  double get() const { return s + c; }
};

// --------------------------------------------------------------- sources
template <class S>
struct Source {
  S Mc, eta, dL, theta, phi, iota, psi, dt, Phic, chi1, chi2, L1, L2;
  S e0;                      // orbital eccentricity at the reference frequency
  double tcoal_days = 0.0;   // GMST of coalescence in sidereal days
  double tc_s = 0.0;         // coalescence time used in the 2 pi f tc phase term [s]
  double f_ref = 0.0;        // reference (GW) frequency of e0 [Hz]
};

// Interferometer geometry; T is the type of the detector parameters.
template <class T>
struct Ifo {
  T lat, lon, gamma;   // radians; gamma = arm-bisector angle from local East
  double zeta;         // opening angle of the arms
  T S0;                // analytic PSD scale [1/Hz], or the scale of a sampled curve
  double f0;           // analytic PSD knee [Hz]
  int site;            // index of the site it belongs to (its noise curve)
};

// Expand sites [lat, lon, gamma, zeta, shape, S0, f0] into interferometers.
// An L site is one interferometer.  A triangle site is three co-located
// interferometers with 60-degree arms in a closed loop (sec. 3.1); the first
// arm points at gamma, so the first interferometer's bisector is at
// gamma + 30 deg and the other two follow at 120 deg steps.  first_site is
// the index of s's first site in the network.
inline std::vector<Ifo<double>> expand_sites(int n_site, const double* s, int first_site = 0) {
  std::vector<Ifo<double>> out;
  for (int i = 0; i < n_site; ++i) {
    const double* r = s + 7 * i;
    if (r[4] == 1.0) {
      for (int k = 0; k < 3; ++k)
        out.push_back({r[0], r[1], r[2] + PI / 6.0 + 2.0 * PI * k / 3.0, PI / 3.0, r[5], r[6], first_site + i});
    } else {
      out.push_back({r[0], r[1], r[2], r[3], r[5], r[6], first_site + i});
    }
  }
  return out;
}

// ----------------------------------------------------------- waveform
// Total mass in seconds and the cut frequency: twice the ISCO orbital
// frequency, i.e. 1/(6^{3/2} pi G M/c^3) (sec. 2.2 footnote).
inline double cut_frequency(double Mc, double eta) {
  double Ms = Mc * std::pow(eta, -0.6) * T_SUN;
  return 1.0 / (std::pow(6.0, 1.5) * PI * Ms);
}

// Tidal combinations of eq. (LamTdelLam_def), sec. 2.1.
template <class S>
void lambda_tilde(const S& eta, const S& L1, const S& L2, S& Lt, S& dLt) {
  using std::sqrt;
  S d = sqrt(1.0 - 4.0 * eta);
  S e2 = eta * eta, e3 = e2 * eta;
  S sum = L1 + L2, dif = L1 - L2;
  Lt = (8.0 / 13.0) * ((1.0 + 7.0 * eta - 31.0 * e2) * sum + d * (1.0 + 9.0 * eta - 11.0 * e2) * dif);
  dLt = 0.5 * (d * (1.0 - (13272.0 / 1319.0) * eta + (8944.0 / 1319.0) * e2) * sum +
               (1.0 - (15910.0 / 1319.0) * eta + (32850.0 / 1319.0) * e2 + (3380.0 / 1319.0) * e3) * dif);
}

// TaylorF2 post-Newtonian phase (without the 2 pi f tc - Phic - pi/4 part),
// 3.5PN point-particle terms with aligned-spin spin-orbit and 2PN spin-spin
// corrections, plus the 5PN/6PN tidal terms (refs. of sec. 2.2).
template <class S>
S pn_phase(const Source<S>& s, const S& v, bool tidal) {
  using std::log; using std::sqrt;
  const double pi = PI, pi2 = PI * PI;
  S eta = s.eta, e2 = eta * eta, e3 = e2 * eta;
  S d = sqrt(1.0 - 4.0 * eta);
  S xs = 0.5 * (s.chi1 + s.chi2), xa = 0.5 * (s.chi1 - s.chi2);
  S lv = log(v);
  S p0 = S(1.0);
  S p2 = 3715.0 / 756.0 + (55.0 / 9.0) * eta;
  S p3 = -16.0 * pi + (113.0 / 3.0) * d * xa + (113.0 / 3.0 - (76.0 / 3.0) * eta) * xs;
  S p4 = 15293365.0 / 508032.0 + (27145.0 / 504.0) * eta + (3085.0 / 72.0) * e2
       + (-405.0 / 8.0 + 200.0 * eta) * xa * xa - (405.0 / 4.0) * d * xa * xs
       + (-405.0 / 8.0 + 2.5 * eta) * xs * xs;
  S p5 = (1.0 + 3.0 * lv) * (pi * (38645.0 / 756.0 - (65.0 / 9.0) * eta)
       - (732985.0 / 2268.0 + (140.0 / 9.0) * eta) * d * xa
       + (-732985.0 / 2268.0 + (24260.0 / 81.0) * eta + (340.0 / 9.0) * e2) * xs);
  S p6 = 11583231236531.0 / 4694215680.0 - (640.0 / 3.0) * pi2 - (6848.0 / 21.0) * EULER_GAMMA
       - (6848.0 / 21.0) * log(4.0 * v)
       + (-15737765635.0 / 3048192.0 + (2255.0 / 12.0) * pi2) * eta
       + (76055.0 / 1728.0) * e2 - (127825.0 / 1296.0) * e3
       + pi * ((2270.0 / 3.0) * d * xa + (2270.0 / 3.0 - 520.0 * eta) * xs);
  S p7 = pi * (77096675.0 / 254016.0 + (378515.0 / 1512.0) * eta - (74045.0 / 756.0) * e2)
       + (-25150083775.0 / 3048192.0 + (26804935.0 / 6048.0) * eta - (1985.0 / 48.0) * e2) * d * xa
       + (-25150083775.0 / 3048192.0 + (10566655595.0 / 762048.0) * eta - (1042165.0 / 3024.0) * e2
          + (5345.0 / 36.0) * e3) * xs;
  S v2 = v * v;
  S series = p0 + v2 * (p2 + v * (p3 + v * (p4 + v * (p5 + v * (p6 + v * p7)))));
  if (tidal) {
    S Lt, dLt;
    lambda_tilde(eta, s.L1, s.L2, Lt, dLt);
    S v10 = v2 * v2 * v2 * v2 * v2;
    series = series + (-19.5) * Lt * v10
           + ((-3115.0 / 64.0) * Lt + (6595.0 / 364.0) * d * dLt) * v10 * v2;
  }
  S v5 = v2 * v2 * v;
  return 3.0 / (128.0 * eta * v5) * series;
}

// Moderate eccentricity (the is_eccentric extension of sec. 2.2, whose
// reference is Moore et al. 2016): to leading order in e0 and at Newtonian
// order, the phase gains -(2355/1462) e0^2 (v_ref/v)^{19/3} times the
// Newtonian term 3/(128 eta v^5), with e0 the eccentricity where the GW
// frequency is f_ref and v_ref = (pi G M f_ref/c^3)^{1/3}.  Valid for
// e0 <~ 0.1 (sec. 2.2).  The numerical coefficient comes from that
// reference, not from the paper.
template <class S>
S eccentric_phase(const Source<S>& s, const S& Ms, const S& v) {
  using std::pow;
  S vref = pow(PI * Ms * s.f_ref, 1.0 / 3.0);
  S v5 = v * v * v * v * v;
  return 3.0 / (128.0 * s.eta * v5) * (-2355.0 / 1462.0) * s.e0 * s.e0 * pow(vref / v, 19.0 / 3.0);
}

// Time to coalescence tau*(f), 3.5PN, non-spinning (the paper cites
// Buonanno et al. 2009, eq. 3.8b, sec. 2.2).
template <class S>
S tau_star(const Source<S>& s, const S& Ms, const S& v) {
  using std::log;
  const double pi = PI, pi2 = PI * PI;
  S eta = s.eta, e2 = eta * eta, e3 = e2 * eta;
  S t2 = 743.0 / 252.0 + (11.0 / 3.0) * eta;
  S t3 = S(-32.0 * pi / 5.0);
  S t4 = 3058673.0 / 508032.0 + (5429.0 / 504.0) * eta + (617.0 / 72.0) * e2;
  S t5 = pi * (-7729.0 / 252.0 + (13.0 / 3.0) * eta);
  S t6 = -10052469856691.0 / 23471078400.0 + (128.0 / 3.0) * pi2 + (6848.0 / 105.0) * EULER_GAMMA
       + (3147553127.0 / 3048192.0 - (451.0 / 12.0) * pi2) * eta
       - (15211.0 / 1728.0) * e2 + (25565.0 / 1296.0) * e3
       + (3424.0 / 105.0) * log(16.0 * v * v);
  S t7 = pi * (-15419335.0 / 127008.0 - (75703.0 / 756.0) * eta + (14809.0 / 378.0) * e2);
  S v2 = v * v;
  S series = 1.0 + v2 * (t2 + v * (t3 + v * (t4 + v * (t5 + v * (t6 + v * t7)))));
  S v8 = v2 * v2 * v2 * v2;
  return 5.0 * Ms / (256.0 * eta * v8) * series;
}

// ------------------------------------------------------ detector response
template <class S> using Vec3 = std::array<S, 3>;
template <class S> S dot(const Vec3<S>& a, const Vec3<S>& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Antenna patterns as tensor contractions F+ = D:e+, Fx = D:ex with the
// detector tensor D = (u u^T - w w^T)/2 built from the unit arm vectors u, w
// at azimuths gamma -/+ zeta/2 (measured from local East towards North) in
// the tangent plane at (lat, local sidereal time lst), and the polarisation
// tensors e+ = X X^T - Y Y^T, ex = X Y^T + Y X^T with X = cos psi e_phi +
// sin psi e_theta, Y = -sin psi e_phi + cos psi e_theta in the equatorial
// frame (sec. 3.1 for gamma and zeta; frame conventions are a reading).
template <class S>
void antenna_tensor(const S& lat, const S& gamma, double zeta, const S& lst,
                    const S& theta, const S& phi, const S& psi, S& Fp, S& Fx) {
  using std::sin; using std::cos;
  S sl = sin(lst), cl = cos(lst), sa = sin(lat), ca = cos(lat);
  Vec3<S> E = {-sl, cl, S(0.0)};
  Vec3<S> N = {-sa * cl, -sa * sl, ca};
  S au = gamma - 0.5 * zeta, aw = gamma + 0.5 * zeta;
  Vec3<S> u, w;
  for (int i = 0; i < 3; ++i) {
    u[i] = cos(au) * E[i] + sin(au) * N[i];
    w[i] = cos(aw) * E[i] + sin(aw) * N[i];
  }
  S st = sin(theta), ct = cos(theta), sp = sin(phi), cp = cos(phi);
  Vec3<S> et = {ct * cp, ct * sp, -st};
  Vec3<S> ep = {-sp, cp, S(0.0)};
  S cs = cos(psi), ss = sin(psi);
  Vec3<S> X, Y;
  for (int i = 0; i < 3; ++i) {
    X[i] = cs * ep[i] + ss * et[i];
    Y[i] = -ss * ep[i] + cs * et[i];
  }
  S fp = S(0.0), fx = S(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S D = 0.5 * (u[i] * u[j] - w[i] * w[j]);
      fp = fp + D * (X[i] * X[j] - Y[i] * Y[j]);
      fx = fx + D * (X[i] * Y[j] + Y[i] * X[j]);
    }
  Fp = fp; Fx = fx;
}

// Arrival-time offset of the interferometer w.r.t. the geocentre:
// -(n . r_det)/c with n the unit vector to the source and r_det the site
// on a spherical Earth (the Doppler term of the Earth-motion footnote).
template <class S>
S geocentre_delay(const S& lat, const S& lst, const S& theta, const S& phi) {
  using std::sin; using std::cos;
  Vec3<S> n = {sin(theta) * cos(phi), sin(theta) * sin(phi), cos(theta)};
  Vec3<S> r = {cos(lat) * cos(lst), cos(lat) * sin(lst), sin(lat)};
  return -(R_EARTH / C_SI) * dot(n, r);
}

// Analytic PSD used by the benchmark networks.
template <class T>
T psd(const T& S0, double f0, double f) {
  double x = f / f0, x2 = x * x;
  double shape = std::pow(x, -4.14) - 5.0 / x2 + 111.0 * (1.0 - x2 + 0.5 * x2 * x2) / (1.0 + 0.5 * x2);
  return S0 * shape;
}

// Sampled noise curves (sec. 3.1: a detector's PSD or ASD read from a file,
// is_ASD telling which): per site, n frequencies f[] (increasing) and values
// S[] there, the PSD itself (kind 1) or the ASD (kind 2), squared into a
// PSD.  The PSD between two samples is the straight line through them (the
// paper does not say how it interpolates; linear in f is the reading).  A
// frequency outside the sampled range is one the detector does not see: its
// point gets no weight.  The end samples are taken to cover frequencies
// within a relative 1e-12 of them, so that a grid starting or ending on a
// sampled frequency keeps that point whatever the rounding of its frequency.
// Set by orc_set_psd_tables for the calls that follow; kind 0 = analytic.
constexpr int MAX_SITES = 8;
static int g_tab_kind[MAX_SITES] = {};
static int64_t g_tab_n[MAX_SITES] = {};
static const double* g_tab_f[MAX_SITES] = {};
static const double* g_tab_S[MAX_SITES] = {};

// The sampled PSD of site i at f (before the scale S0); false outside the range.
inline bool table_psd(int i, double f, double& S) {
  const int64_t n = g_tab_n[i];
  const double* tf = g_tab_f[i];
  const double* tS = g_tab_S[i];
  const double eps = 1e-12;
  if (f < tf[0] * (1.0 - eps) || f > tf[n - 1] * (1.0 + eps)) return false;
  // the interval [tf[j], tf[j+1]] holding f (the first or last one at the ends):
  // j is the last sample at or below f
  int64_t j = (int64_t)(std::upper_bound(tf, tf + n, f) - tf) - 1;
  if (j < 0) j = 0;
  if (j > n - 2) j = n - 2;
  double s0 = tS[j], s1 = tS[j + 1];
  if (g_tab_kind[i] == 2) {
    s0 = s0 * s0;
    s1 = s1 * s1;
  }
  double t = (f - tf[j]) / (tf[j + 1] - tf[j]);
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  S = s0 + (s1 - s0) * t;
  return true;
}

// The noise weight 4 w / S_n(f) of one interferometer at a grid point of
// trapezoid weight w (zero where a sampled curve does not reach).
template <class T>
T noise_weight(const Ifo<T>& ifo, double w, double f) {
  const int i = ifo.site;
  if (i >= 0 && i < MAX_SITES && g_tab_kind[i] != 0) {
    double S;
    if (!table_psd(i, f, S)) return T(0.0);
    return T(4.0 * w) / (ifo.S0 * S);
  }
  return T(4.0 * w) / psd(ifo.S0, ifo.f0, f);
}

// Strain h_i(f) at one interferometer: restricted amplitude (Newtonian
// order, sqrt(5/24) pi^{-2/3} (G Mc/c^3)^{5/6} f^{-7/6} c/dL) times the
// pattern-weighted polarisations, h+ ~ (1+cos^2 iota)/2, hx ~ i cos iota,
// with the phase Psi = 2 pi f (tc + dt + Delta) - Phic - pi/4 + Psi_PN.
template <class S, class T>
void strain(const Source<S>& s, const Ifo<T>& ifo, double f, int flags, S& hre, S& him) {
  using std::sin; using std::cos; using std::pow; using std::sqrt;
  S Ms = s.Mc * pow(s.eta, -0.6) * T_SUN;
  S v = pow(PI * Ms * f, 1.0 / 3.0);
  S tau = tau_star(s, Ms, v);
  // GMST at t(f): 2 pi tcoal + Omega (dt - tau*(f)); without rotation the
  // patterns are frozen at the coalescence time.
  S thG = (flags & FLAG_EARTH_ROT) ? (2.0 * PI * s.tcoal_days + OMEGA_E * (s.dt - tau))
                                   : (2.0 * PI * s.tcoal_days + OMEGA_E * s.dt);
  S lat = lift<S>(ifo.lat), lon = lift<S>(ifo.lon), gam = lift<S>(ifo.gamma);
  S lst = thG + lon;
  S Fp, Fx;
  antenna_tensor(lat, gam, ifo.zeta, lst, s.theta, s.phi, s.psi, Fp, Fx);
  S Delta = geocentre_delay(lat, lst, s.theta, s.phi);
  S ci = cos(s.iota);
  S amp = (sqrt(5.0 / 24.0) * pow(PI, -2.0 / 3.0)) * pow(s.Mc * T_SUN, 5.0 / 6.0) * pow(f, -7.0 / 6.0) /
          (s.dL * GPC_S);
  S qre = amp * Fp * 0.5 * (1.0 + ci * ci);
  S qim = amp * Fx * ci;
  S Psi = 2.0 * PI * f * (s.tc_s + s.dt + Delta) - s.Phic - 0.25 * PI + pn_phase(s, v, (flags & FLAG_TIDAL) != 0);
  if (flags & FLAG_ECC) Psi = Psi + eccentric_phase(s, Ms, v);
  S c = cos(Psi), sn = sin(Psi);
  hre = qre * c - qim * sn;
  him = qre * sn + qim * c;
}

// ------------------------------------------------------------------ grid
// Log-spaced grid with fixed end points, as numpy's geomspace builds it
// (sec. 2.2 example): f_k = fmin exp(k D), D = ln(fmax/fmin)/(n-1), with
// f_0 = fmin and f_{n-1} = fmax exactly.  Trapezoid weights, literally:
// w_0 = (f_1-f_0)/2, w_k = (f_{k+1}-f_{k-1})/2, w_{n-1} = (f_{n-1}-f_{n-2})/2.
inline void make_grid(double fmin, double fmax, int n, std::vector<double>& f, std::vector<double>& w) {
  f.assign(n, 0.0);
  w.assign(n, 0.0);
  double D = std::log(fmax / fmin) / (n - 1);
  for (int k = 0; k < n; ++k) f[k] = fmin * std::exp(k * D);
  f[0] = fmin;
  f[n - 1] = fmax;
  for (int k = 0; k < n; ++k) {
    double hi = f[k < n - 1 ? k + 1 : k], lo = f[k > 0 ? k - 1 : k];
    w[k] = 0.5 * (hi - lo);
  }
}

// An explicit grid (the frequencies themselves, event e's at off[e] ..
// off[e] + npts[e] - 1 of f) in place of the log descriptors, for the
// workload-level drivers below; set by orc_set_explicit_grid, NULL = none.
static const int64_t* g_grid_off = nullptr;
static const double* g_grid_f = nullptr;

// Event e's grid and trapezoid weights: the explicit frequencies if set,
// else the log grid from fmin to fhi.
inline void event_grid(int64_t e, double fmin, double fhi, int n, std::vector<double>& f,
                       std::vector<double>& w) {
  if (!g_grid_f || e < 0) {
    make_grid(fmin, fhi, n, f, w);
    return;
  }
  f.assign(g_grid_f + g_grid_off[e], g_grid_f + g_grid_off[e] + n);
  w.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double hi = f[k < n - 1 ? k + 1 : k], lo = f[k > 0 ? k - 1 : k];
    w[k] = 0.5 * (hi - lo);
  }
}

// ----------------------------------------------------- per-event sums
template <class S>
Source<S> make_source(const double* par, double tc_s) {
  Source<S> s;
  s.Mc = S(par[0]); s.eta = S(par[1]); s.dL = S(par[2]); s.theta = S(par[3]);
  s.phi = S(par[4]); s.iota = S(par[5]); s.psi = S(par[6]); s.dt = S(0.0);
  s.Phic = S(par[8]); s.chi1 = S(par[9]); s.chi2 = S(par[10]);
  s.L1 = S(par[11]); s.L2 = S(par[12]);
  s.e0 = S(par[13]);
  s.tcoal_days = par[7];
  s.tc_s = tc_s;
  s.f_ref = par[14];
  return s;
}

// Number of Fisher parameters: 11, plus the two deformabilities, plus e0.
inline int n_params(int flags) {
  return 11 + ((flags & FLAG_TIDAL) ? 2 : 0) + ((flags & FLAG_ECC) ? 1 : 0);
}

// Per-event eccentricities and their reference frequencies for the
// workload-level drivers (orc_set_eccentricity); NULL = none / the grid's
// first frequency.
static const double* g_ecc = nullptr;
static const double* g_fref = nullptr;

// Event e's parameters: the 13 rows of par, then e0 and f_ref (0 = the
// grid's first frequency).
inline void event_params(const double* par, int64_t ld, int64_t e, double* p) {
  for (int i = 0; i < 13; ++i) p[i] = par[i * ld + e];
  p[13] = g_ecc ? g_ecc[e] : 0.0;
  p[14] = g_fref ? g_fref[e] : 0.0;
}

// Slot i of the Fisher matrix, in the parameter order of the public tables
// (sec. 3.2): e0 comes after the spins and the deformabilities.
template <class S>
S& slot(Source<S>& s, int i, int flags) {
  if ((flags & FLAG_ECC) && i == n_params(flags) - 1) return s.e0;
  switch (i) {
    case 0: return s.Mc; case 1: return s.eta; case 2: return s.dL; case 3: return s.theta;
    case 4: return s.phi; case 5: return s.iota; case 6: return s.psi; case 7: return s.dt;
    case 8: return s.Phic; case 9: return s.chi1; case 10: return s.chi2; case 11: return s.L1;
    default: return s.L2;
  }
}

// SNR^2 per interferometer and Fisher per interferometer (optional) for one
// event, derivatives by Dual<double,P>; all sums compensated.
template <int P>
void fisher_event(const double* par, double tc_s, const std::vector<Ifo<double>>& ifos,
                  double fmin, double fmax, int n, int flags,
                  double* snr2_ifo, double* F_ifo /* [n_ifo][P][P] */, int64_t e = -1) {
  using S = Dual<double, P>;
  Source<S> s = make_source<S>(par, tc_s);
  for (int i = 0; i < P; ++i) slot(s, i, flags).d[i] = 1.0;
  std::vector<double> f, w;
  event_grid(e, fmin, fmax, n, f, w);
  if (!(s.f_ref > 0.0)) s.f_ref = f[0];   // e0 given at the grid's first frequency
  const int nifo = (int)ifos.size();
  for (int d = 0; d < nifo; ++d) {
    NeumaierSum snr;
    std::vector<NeumaierSum> G(P * P);
    for (int k = 0; k < n; ++k) {
      S hre, him;
      strain(s, ifos[d], f[k], flags, hre, him);
      double om = noise_weight(ifos[d], w[k], f[k]);
      snr.add(om * (hre.v * hre.v + him.v * him.v));
      for (int a = 0; a < P; ++a)
        for (int b = a; b < P; ++b)
          G[a * P + b].add(om * (hre.d[a] * hre.d[b] + him.d[a] * him.d[b]));
    }
    snr2_ifo[d] = snr.get();
    for (int a = 0; a < P; ++a)
      for (int b = a; b < P; ++b) {
        double g = G[a * P + b].get();
        F_ifo[(d * P + a) * P + b] = g;
        F_ifo[(d * P + b) * P + a] = g;
      }
  }
}

// Network SNR^2 and Fisher matrix of one event together with their
// derivatives along one detector parameter: the detector parameters carry a
// one-component dual number (type D1) inside the P-component dual numbers of
// the source parameters, so every strain derivative d_i h also carries its
// own derivative along the detector parameter.  Plain sums of values and of
// tangents, each compensated.
using D1 = Dual<double, 1>;

template <int P>
void fisher_event_tangent(const double* par, double tc_s, const std::vector<Ifo<D1>>& ifos,
                          const std::vector<char>& on, double fmin, double fmax, int n, int flags,
                          double* snr2 /* [2] */, double* F /* [2][P][P] */, int64_t e = -1) {
  using S = Dual<D1, P>;
  Source<S> s = make_source<S>(par, tc_s);
  for (int i = 0; i < P; ++i) slot(s, i, flags).d[i] = D1(1.0);
  std::vector<double> f, w;
  event_grid(e, fmin, fmax, n, f, w);
  if (!(s.f_ref > 0.0)) s.f_ref = f[0];   // e0 given at the grid's first frequency
  NeumaierSum sv, st;
  std::vector<NeumaierSum> Gv(P * P), Gt(P * P);
  for (size_t d = 0; d < ifos.size(); ++d)
    for (int k = 0; k < n; ++k) {
      if (!on[d]) break;                       // interferometer off for this event
      S hre, him;
      strain(s, ifos[d], f[k], flags, hre, him);
      D1 om = noise_weight(ifos[d], w[k], f[k]);
      D1 a = om * (hre.v * hre.v + him.v * him.v);
      sv.add(a.v); st.add(a.d[0]);
      for (int i = 0; i < P; ++i)
        for (int j = i; j < P; ++j) {
          D1 g = om * (hre.d[i] * hre.d[j] + him.d[i] * him.d[j]);
          Gv[i * P + j].add(g.v); Gt[i * P + j].add(g.d[0]);
        }
    }
  snr2[0] = sv.get(); snr2[1] = st.get();
  for (int i = 0; i < P; ++i)
    for (int j = i; j < P; ++j) {
      F[i * P + j] = F[j * P + i] = Gv[i * P + j].get();
      F[P * P + i * P + j] = F[P * P + j * P + i] = Gt[i * P + j].get();
    }
}

void snr_event(const double* par, double tc_s, const std::vector<Ifo<double>>& ifos, double fmin,
               double fmax, int n, int flags, double* snr2_ifo, int64_t e = -1) {
  Source<double> s = make_source<double>(par, tc_s);
  std::vector<double> f, w;
  event_grid(e, fmin, fmax, n, f, w);
  if (!(s.f_ref > 0.0)) s.f_ref = f[0];   // e0 given at the grid's first frequency
  for (size_t d = 0; d < ifos.size(); ++d) {
    NeumaierSum snr;
    for (int k = 0; k < n; ++k) {
      double hre, him;
      strain(s, ifos[d], f[k], flags, hre, him);
      snr.add(noise_weight(ifos[d], w[k], f[k]) * (hre * hre + him * him));
    }
    snr2_ifo[d] = snr.get();
  }
}

}  // namespace orc

// =================================================================== C API
using namespace orc;

// Strain derivatives of n events with respect to their P parameters (the
// Fisher matrix's rows and units), by forward-mode dual numbers through the
// same strain as orc_waveform: dh[P][n_ifo][total][2], event e at columns
// offsets[e] .. offsets[e] + npts[e] - 1.
template <int P>
static void waveform_deriv_events(int64_t n, const double* par, int64_t ld, const double* tc_s,
                                  const std::vector<Ifo<double>>& ifos, const double* fmin,
                                  const double* fmax, const int32_t* npts, int flags,
                                  const int64_t* offsets, int64_t total, double* dh) {
  using S = Dual<double, P>;
  const int nifo = (int)ifos.size();
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n; ++e) {
    double p[15];
    event_params(par, ld, e, p);
    double fhi = fmax ? fmax[e] : cut_frequency(p[0], p[1]);
    Source<S> s = make_source<S>(p, tc_s ? tc_s[e] : 0.0);
    for (int j = 0; j < P; ++j) slot(s, j, flags).d[j] = 1.0;
    std::vector<double> f, w;
    event_grid(e, fmin[e], fhi, npts[e], f, w);
    if (!(s.f_ref > 0.0)) s.f_ref = f[0];
    for (int d = 0; d < nifo; ++d)
      for (int k = 0; k < npts[e]; ++k) {
        S hr, hi;
        strain(s, ifos[d], f[k], flags, hr, hi);
        for (int j = 0; j < P; ++j) {
          double* o = dh + (((int64_t)j * nifo + d) * total + offsets[e] + k) * 2;
          o[0] = hr.d[j];
          o[1] = hi.d[j];
        }
      }
  }
}

template <int P>
static void strain_events_one(const double* par, double tc_s, const std::vector<Ifo<double>>& ifos, int nf,
                              const double* f, int flags, double* h, double* dh) {
  using S = Dual<double, P>;
  for (size_t i = 0; i < ifos.size(); ++i)
    for (int k = 0; k < nf; ++k) {
      Source<S> s = make_source<S>(par, tc_s);
      if (!(s.f_ref > 0.0)) s.f_ref = f[0];
      for (int j = 0; j < P; ++j) slot(s, j, flags).d[j] = 1.0;
      S hr, hi;
      strain(s, ifos[i], f[k], flags, hr, hi);
      h[(i * nf + k) * 2] = hr.v; h[(i * nf + k) * 2 + 1] = hi.v;
      if (dh) for (int j = 0; j < P; ++j) {
        dh[((i * nf + k) * P + j) * 2] = hr.d[j]; dh[((i * nf + k) * P + j) * 2 + 1] = hi.d[j];
      }
    }
}

extern "C" {

// Constants, for the record of what the oracle assumed.
void orc_constants(double* out /* [6] */) {
  out[0] = T_SUN; out[1] = GPC_S; out[2] = OMEGA_E; out[3] = R_EARTH / C_SI; out[4] = EULER_GAMMA; out[5] = PI;
}

double orc_cut_frequency(double Mc, double eta) { return cut_frequency(Mc, eta); }
double orc_psd(double S0, double f0, double f) { return psd(S0, f0, f); }

void orc_grid(double fmin, double fmax, int n, double* f, double* w) {
  std::vector<double> ff, ww;
  make_grid(fmin, fmax, n, ff, ww);
  std::memcpy(f, ff.data(), n * sizeof(double));
  std::memcpy(w, ww.data(), n * sizeof(double));
}

int orc_n_ifo(int n_site, const double* sites) { return (int)expand_sites(n_site, sites).size(); }

// Interferometer geometry after expanding triangles: [n_ifo][4] = lat, lon, gamma, zeta.
void orc_ifos(int n_site, const double* sites, double* out) {
  auto v = expand_sites(n_site, sites);
  for (size_t i = 0; i < v.size(); ++i) {
    out[4 * i] = v[i].lat; out[4 * i + 1] = v[i].lon; out[4 * i + 2] = v[i].gamma; out[4 * i + 3] = v[i].zeta;
  }
}

void orc_antenna(double lat, double gamma, double zeta, double lst, double theta, double phi,
                 double psi, double* Fp, double* Fx) {
  antenna_tensor(lat, gamma, zeta, lst, theta, phi, psi, *Fp, *Fx);
}

double orc_delay(double lat, double lst, double theta, double phi) {
  return geocentre_delay(lat, lst, theta, phi);
}

// PN phase and tau*(f) of one event on nf frequencies.
void orc_phase_tau(const double* par, int flags, int nf, const double* f, double* psi_pn, double* tau) {
  Source<double> s = make_source<double>(par, 0.0);
  if (!(s.f_ref > 0.0)) s.f_ref = f[0];
  double Ms = s.Mc * std::pow(s.eta, -0.6) * T_SUN;
  for (int k = 0; k < nf; ++k) {
    double v = std::pow(PI * Ms * f[k], 1.0 / 3.0);
    psi_pn[k] = pn_phase(s, v, (flags & FLAG_TIDAL) != 0);
    if (flags & FLAG_ECC) psi_pn[k] += eccentric_phase(s, Ms, v);
    tau[k] = tau_star(s, Ms, v);
  }
}

// Complex-step derivative of the PN phase (with the eccentric term under
// FLAG_ECC) with respect to parameter slot j at fixed frequency:
// Im Psi(par + i h e_j) / h.
void orc_phase_cstep_par(const double* par, int flags, int j, int nf, const double* f, double h, double* out) {
  using C = std::complex<double>;
  Source<C> s = make_source<C>(par, 0.0);
  if (!(s.f_ref > 0.0)) s.f_ref = f[0];
  slot(s, j, flags) = slot(s, j, flags) + C(0.0, h);
  C Ms = s.Mc * std::pow(s.eta, -0.6) * T_SUN;
  for (int k = 0; k < nf; ++k) {
    C v = std::pow(PI * Ms * f[k], 1.0 / 3.0);
    C psi = pn_phase(s, v, (flags & FLAG_TIDAL) != 0);
    if (flags & FLAG_ECC) psi = psi + eccentric_phase(s, Ms, v);
    out[k] = psi.imag() / h;
  }
}

// Eccentricities e0[n] and reference frequencies f_ref[n] (NULL: each grid's
// first frequency) of the workload-level drivers that follow; NULL, NULL
// clears them.  The arrays must stay alive while they are set.
int orc_set_eccentricity(const double* e0, const double* f_ref) {
  g_ecc = e0;
  g_fref = f_ref;
  return 0;
}

// Complex-step version of the PN phase: Im(Psi(f + i h))/h = dPsi/df.
void orc_phase_cstep_f(const double* par, int flags, int nf, const double* f, double h, double* dpsi_df) {
  using C = std::complex<double>;
  Source<C> s = make_source<C>(par, 0.0);
  C Ms = s.Mc * std::pow(s.eta, -0.6) * T_SUN;
  for (int k = 0; k < nf; ++k) {
    C v = std::pow(PI * Ms * C(f[k], h), 1.0 / 3.0);
    dpsi_df[k] = pn_phase(s, v, (flags & FLAG_TIDAL) != 0).imag() / h;
  }
}

// Strain of one event at every interferometer on an explicit frequency list,
// h[(i*nf + k)*2 + {0,1}], and optionally its P derivatives by dual numbers,
// dh[((i*nf + k)*P + j)*2 + {0,1}].  par holds the 13 parameters, e0 and
// f_ref (0: the list's first frequency).
int orc_strain(const double* par, double tc_s, int n_site, const double* sites, int nf,
               const double* f, int flags, double* h, double* dh) {
  auto ifos = expand_sites(n_site, sites);
  switch (n_params(flags)) {
    case 14: strain_events_one<14>(par, tc_s, ifos, nf, f, flags, h, dh); break;
    case 13: strain_events_one<13>(par, tc_s, ifos, nf, f, flags, h, dh); break;
    case 12: strain_events_one<12>(par, tc_s, ifos, nf, f, flags, h, dh); break;
    default: strain_events_one<11>(par, tc_s, ifos, nf, f, flags, h, dh);
  }
  return 0;
}

// Complex-step derivative of the strain w.r.t. parameter slot j (slot 7 is
// the coalescence-time shift in seconds): dh = Im h(par + i step e_j)/step,
// applied to the real and the imaginary part of h separately.
int orc_strain_cstep(const double* par, double tc_s, int n_site, const double* sites, int nf,
                     const double* f, int flags, int j, double step, double* dh) {
  using C = std::complex<double>;
  auto ifos = expand_sites(n_site, sites);
  Source<C> s = make_source<C>(par, tc_s);
  if (!(s.f_ref > 0.0)) s.f_ref = f[0];
  slot(s, j, flags) = slot(s, j, flags) + C(0.0, step);
  for (size_t i = 0; i < ifos.size(); ++i)
    for (int k = 0; k < nf; ++k) {
      C hr, hi;
      strain(s, ifos[i], f[k], flags, hr, hi);
      dh[(i * nf + k) * 2] = hr.imag() / step;
      dh[(i * nf + k) * 2 + 1] = hi.imag() / step;
    }
  return 0;
}

// Plain strain (double) with the coalescence-time slot shifted by dt seconds
// and the other slots as given; used for finite-difference checks.
int orc_strain_plain(const double* par, double tc_s, double dt, int n_site, const double* sites,
                     int nf, const double* f, int flags, double* h) {
  auto ifos = expand_sites(n_site, sites);
  Source<double> s = make_source<double>(par, tc_s);
  if (!(s.f_ref > 0.0)) s.f_ref = f[0];
  s.dt = dt;
  for (size_t i = 0; i < ifos.size(); ++i)
    for (int k = 0; k < nf; ++k) strain(s, ifos[i], f[k], flags, h[(i * nf + k) * 2], h[(i * nf + k) * 2 + 1]);
  return 0;
}

// Strain of n events at every interferometer on each event's own log grid
// (the detector strain of sec. 3.1 on the grids of sec. 2.2), written to
// h[((i * total) + offsets[e] + k) * 2 + {0,1}] for interferometer i, grid
// point k (offsets[n] are the events' first columns).  fmax NULL means each grid ends at the event's cut frequency.
// Sampled noise curves of the sites (see table_psd) for the calls that
// follow: kind[i] 0 (analytic), 1 (PSD) or 2 (ASD) for site i, and for the
// sampled ones n[i] frequencies f[i][] with values S[i][]; n_site = 0
// clears them.  The arrays must stay alive while they are set.
int orc_set_psd_tables(int n_site, const int32_t* kind, const int64_t* n, const double* const* f,
                       const double* const* S) {
  for (int i = 0; i < MAX_SITES; ++i) {
    const bool set = i < n_site && kind && kind[i] != 0;
    g_tab_kind[i] = set ? kind[i] : 0;
    g_tab_n[i] = set ? n[i] : 0;
    g_tab_f[i] = set ? f[i] : nullptr;
    g_tab_S[i] = set ? S[i] : nullptr;
  }
  return 0;
}

// The noise weight of an L site's interferometer (site 0 of the tables set)
// or of the analytic PSD at frequencies f with trapezoid weights w.
void orc_noise_weight(double S0, double f0, int site, int nf, const double* f, const double* w, double* out) {
  Ifo<double> g{0.0, 0.0, 0.0, 0.0, S0, f0, site};
  for (int k = 0; k < nf; ++k) out[k] = noise_weight(g, w[k], f[k]);
}

int orc_set_explicit_grid(const int64_t* off, const double* f) {
  g_grid_off = off;
  g_grid_f = f;
  return 0;
}

int orc_waveform(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site,
                 const double* sites, const double* fmin, const double* fmax, const int32_t* npts,
                 int flags, int nthreads, const int64_t* offsets, int64_t total, double* h) {
  auto ifos = expand_sites(n_site, sites);
  const int nifo = (int)ifos.size();
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n; ++e) {
    double p[15];
    event_params(par, ld, e, p);
    double fhi = fmax ? fmax[e] : cut_frequency(p[0], p[1]);
    Source<double> s = make_source<double>(p, tc_s ? tc_s[e] : 0.0);
    std::vector<double> f, w;
    event_grid(e, fmin[e], fhi, npts[e], f, w);
    if (!(s.f_ref > 0.0)) s.f_ref = f[0];
    for (int d = 0; d < nifo; ++d)
      for (int k = 0; k < npts[e]; ++k) {
        double* o = h + ((int64_t)d * total + offsets[e] + k) * 2;
        strain(s, ifos[d], f[k], flags, o[0], o[1]);
      }
  }
  return 0;
}

int orc_waveform_deriv(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site,
                       const double* sites, const double* fmin, const double* fmax,
                       const int32_t* npts, int flags, int nthreads, const int64_t* offsets,
                       int64_t total, double* dh) {
  auto ifos = expand_sites(n_site, sites);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  switch (n_params(flags)) {
    case 14: waveform_deriv_events<14>(n, par, ld, tc_s, ifos, fmin, fmax, npts, flags, offsets, total, dh); break;
    case 13: waveform_deriv_events<13>(n, par, ld, tc_s, ifos, fmin, fmax, npts, flags, offsets, total, dh); break;
    case 12: waveform_deriv_events<12>(n, par, ld, tc_s, ifos, fmin, fmax, npts, flags, offsets, total, dh); break;
    default: waveform_deriv_events<11>(n, par, ld, tc_s, ifos, fmin, fmax, npts, flags, offsets, total, dh);
  }
  return 0;
}

// SNR^2 and Fisher matrix of n events and their derivatives along one
// detector parameter: parameter `which` (0 latitude, 1 longitude, 2 arm angle
// gamma, 3 ln S0) of site `site`.  Outputs snr2[2][n] (value, derivative)
// and fisher[2][P][P][n].
int orc_fisher_tangent(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site,
                       const double* sites, const double* fmin, const double* fmax,
                       const int32_t* npts, const uint8_t* active, int flags, int nthreads, int site,
                       int which, double* snr2, double* fisher) {
  std::vector<Ifo<D1>> ifos;
  for (int i = 0; i < n_site; ++i) {
    const double* r = sites + 7 * i;
    const double seed = (i == site) ? 1.0 : 0.0;
    for (const Ifo<double>& g : expand_sites(1, r, i)) {
      Ifo<D1> t;
      t.lat = D1(g.lat); t.lon = D1(g.lon); t.gamma = D1(g.gamma); t.zeta = g.zeta;
      t.S0 = D1(g.S0); t.f0 = g.f0; t.site = g.site;
      if (which == 0) t.lat.d[0] = seed;
      if (which == 1) t.lon.d[0] = seed;
      if (which == 2) t.gamma.d[0] = seed;
      if (which == 3) t.S0.d[0] = seed * g.S0;       // dS0 / d ln S0
      ifos.push_back(t);
    }
  }
  const int P = n_params(flags);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n; ++e) {
    double p[15];
    event_params(par, ld, e, p);
    double fhi = fmax ? fmax[e] : cut_frequency(p[0], p[1]);
    double tcs = tc_s ? tc_s[e] : 0.0;
    double s2[2];
    std::vector<double> F(2 * P * P);
    std::vector<char> on(ifos.size(), 1);
    if (active)
      for (size_t d = 0; d < ifos.size(); ++d) on[d] = active[(int64_t)d * n + e] != 0;
    switch (P) {
      case 14: fisher_event_tangent<14>(p, tcs, ifos, on, fmin[e], fhi, npts[e], flags, s2, F.data(), e); break;
      case 13: fisher_event_tangent<13>(p, tcs, ifos, on, fmin[e], fhi, npts[e], flags, s2, F.data(), e); break;
      case 12: fisher_event_tangent<12>(p, tcs, ifos, on, fmin[e], fhi, npts[e], flags, s2, F.data(), e); break;
      default: fisher_event_tangent<11>(p, tcs, ifos, on, fmin[e], fhi, npts[e], flags, s2, F.data(), e);
    }
    snr2[e] = s2[0];
    snr2[n + e] = s2[1];
    for (int t = 0; t < 2; ++t)
      for (int a = 0; a < P * P; ++a) fisher[((int64_t)t * P * P + a) * n + e] = F[t * P * P + a];
  }
  return 0;
}

// SNR and Fisher matrices of n events (parameters [13][ld], event fastest).
// Outputs (any may be NULL except snr):
//   snr[n]; snr_ifo[n_ifo][n] (SNR of each interferometer);
//   fisher[P][P][n] network Fisher; fisher_ifo[n_ifo][P][P][n].
// fmax NULL means each grid ends at the event's cut frequency.  active
// [n_ifo][n] (NULL: all on): interferometers off for an event (the duty
// factor) are left out of its network sums and report zero.
int orc_fisher(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site,
               const double* sites, const double* fmin, const double* fmax, const int32_t* npts,
               const uint8_t* active, int flags, int nthreads, double* snr, double* snr_ifo,
               double* fisher, double* fisher_ifo) {
  auto ifos = expand_sites(n_site, sites);
  const int nifo = (int)ifos.size();
  const int P = n_params(flags);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < n; ++e) {
    double p[15];
    event_params(par, ld, e, p);
    double fhi = fmax ? fmax[e] : cut_frequency(p[0], p[1]);
    double tcs = tc_s ? tc_s[e] : 0.0;
    std::vector<double> s2(nifo), F;
    if (fisher || fisher_ifo) {
      F.assign((size_t)nifo * P * P, 0.0);
      switch (P) {
        case 14: fisher_event<14>(p, tcs, ifos, fmin[e], fhi, npts[e], flags, s2.data(), F.data(), e); break;
        case 13: fisher_event<13>(p, tcs, ifos, fmin[e], fhi, npts[e], flags, s2.data(), F.data(), e); break;
        case 12: fisher_event<12>(p, tcs, ifos, fmin[e], fhi, npts[e], flags, s2.data(), F.data(), e); break;
        default: fisher_event<11>(p, tcs, ifos, fmin[e], fhi, npts[e], flags, s2.data(), F.data(), e);
      }
    } else {
      snr_event(p, tcs, ifos, fmin[e], fhi, npts[e], flags, s2.data(), e);
    }
    if (active)
      for (int d = 0; d < nifo; ++d)
        if (!active[(int64_t)d * n + e]) {
          s2[d] = 0.0;
          if (!F.empty()) std::fill(F.begin() + (size_t)d * P * P, F.begin() + (size_t)(d + 1) * P * P, 0.0);
        }
    NeumaierSum tot;
    for (int d = 0; d < nifo; ++d) tot.add(s2[d]);
    snr[e] = std::sqrt(tot.get());
    if (snr_ifo) for (int d = 0; d < nifo; ++d) snr_ifo[d * n + e] = std::sqrt(s2[d]);
    if (fisher)
      for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) {
          NeumaierSum g;
          for (int d = 0; d < nifo; ++d) g.add(F[((size_t)d * P + a) * P + b]);
          fisher[((int64_t)a * P + b) * n + e] = g.get();
        }
    if (fisher_ifo)
      for (int d = 0; d < nifo; ++d)
        for (int a = 0; a < P * P; ++a) fisher_ifo[((int64_t)d * P * P + a) * n + e] = F[(size_t)d * P * P + a];
  }
  return 0;
}

}  // extern "C"

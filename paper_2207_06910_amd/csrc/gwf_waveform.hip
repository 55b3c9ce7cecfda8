// gwf_waveform.hip -- the strain itself at every interferometer and grid
// point (the paper's GWstrain, sec. 3.1):
//   h_i(f) = A(f) [F+_i (1+cos^2 iota)/2 + i Fx_i cos iota] exp(i Psi_i),
//   Psi_i  = 2 pi f (tc + Delta_i) - Phic - pi/4 + Psi_PN(f),
// with the patterns and the arrival-time offset Delta_i at t(f) when the
// Earth rotates.  Unlike SNR and Fisher this needs the phase itself, which
// reaches ~1e7 rad at a few Hz for neutron-star binaries and 2 pi f tc for
// GPS-scale tc; the phase is therefore assembled in cycles, each term
// reduced to its fractional part (f tc from the exact product inside a fused
// multiply-add), and only the final fraction in [-1/2, 1/2] goes through
// sin/cos.
//
// One workgroup per event, lanes over grid points: each interferometer's
// output row is written with consecutive lanes on consecutive 16-byte
// complex values, so the kernel streams its output at HBM rate.
#include "gwf_kernels.hpp"

namespace gwf {

namespace {

constexpr int kWBlock = 256;

// Per-site constants of the strain loop: rotation to the site's hour angle,
// the delay, and for each computed arm the projected amplitude's real and
// imaginary parts (c+ F+ and cx Fx, inclination factors folded in) as
// trigonometric polynomials in the hour angle H: coefficients of
// (1, cos H, sin H, cos 2H, sin 2H).
struct WaveSite {
  double cdl, sdl, k1, k0;
  double m[2][2][5];
  int32_t n_arm, pad;
};

__device__ inline double trig5(const double c[5], double cH, double sH, double c2H, double s2H) {
  return fma(c[4], s2H, fma(c[3], c2H, fma(c[2], sH, c[1] * cH))) + c[0];
}

// Event e's inputs: the 13 parameters (no tidal rows without tides), e0 and
// its reference frequency (with the eccentric flag, else zero).
__device__ inline void load_event(const WaveformArgs& a, int64_t e, bool tidal, double* p) {
  for (int r = 0; r < 13; ++r) p[r] = (r < 11 || tidal) ? a.par[r * a.ld + e] : 0.0;
  p[13] = a.ecc_flag && a.ecc ? a.ecc[e] : 0.0;
  p[14] = a.ecc_flag && a.fref ? a.fref[e] : 0.0;
}

// x reduced to [-1/2, 1/2] by subtracting the nearest integer (exact).
__device__ inline double frac_center(double x) { return x - rint(x); }

// sin and cos of 2 pi x for |x| <= 1/2.  FP64: the quarter-turn q = rint(4x)
// and the rest r = x - q/4 are exact in cycles (|r| <= 1/8), so t = 2 pi r
// carries one rounding (|t| <= pi/4) and needs no Cody-Waite reduction; the
// Taylor series of sin to t^17 and cos to t^16 truncate below 1e-18.
// Mixed form: the quarter-turn q = rint(4x) and the rest
// r = x - q/4 (exact, |r| <= 1/8) are taken in FP64, then the Taylor series
// of sin (to the 9th power) and cos (to the 10th) of 2 pi r in FP32, whose
// truncation errors (< 2e-9, < 2e-10 on |2 pi r| <= pi/4) lie below the
// FP32 rounding; the absolute error is a few 1e-8 rad from rounding r and
// about 1e-7 from the FP32 arithmetic.
template <bool MIXED>
__device__ inline void sincos_cycles(double x, double* s, double* c) {
  if (MIXED) {
    const double q = rint(4.0 * x);
    const float t = (float)kTwoPi * (float)fma(-0.25, q, x);
    const float t2 = t * t;
    float ps = fmaf(t2, 1.0f / 362880.0f, -1.0f / 5040.0f);
    ps = fmaf(ps, t2, 1.0f / 120.0f);
    ps = fmaf(ps, t2, -1.0f / 6.0f);
    const float sr = fmaf(t * t2, ps, t);
    float pc = fmaf(t2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    pc = fmaf(pc, t2, -1.0f / 720.0f);
    pc = fmaf(pc, t2, 1.0f / 24.0f);
    pc = fmaf(pc, t2, -0.5f);
    const float cr = fmaf(t2, pc, 1.0f);
    const int k = (int)q & 3;                  // angle = k quarter turns + t
    const float ss = (k & 1) ? cr : sr, cc = (k & 1) ? sr : cr;
    *s = (double)((k & 2) ? -ss : ss);
    *c = (double)(((k + 1) & 2) ? -cc : cc);
  } else {
    const double q = rint(4.0 * x);
    const double t = kTwoPi * fma(-0.25, q, x);
    const double t2 = t * t;
    double ps = -1.0 / 355687428096000.0;          // -1/17!
    ps = fma(ps, t2, 1.0 / 1307674368000.0);       //  1/15!
    ps = fma(ps, t2, -1.0 / 6227020800.0);         // -1/13!
    ps = fma(ps, t2, 1.0 / 39916800.0);            //  1/11!
    ps = fma(ps, t2, -1.0 / 362880.0);             // -1/9!
    ps = fma(ps, t2, 1.0 / 5040.0);                //  1/7!
    ps = fma(ps, t2, -1.0 / 120.0);                // -1/5!
    ps = fma(ps, t2, 1.0 / 6.0);                   //  1/3!
    const double sr = fma(-t * t2, ps, t);
    double pc = 1.0 / 20922789888000.0;            //  1/16!
    pc = fma(pc, t2, -1.0 / 87178291200.0);        // -1/14!
    pc = fma(pc, t2, 1.0 / 479001600.0);           //  1/12!
    pc = fma(pc, t2, -1.0 / 3628800.0);            // -1/10!
    pc = fma(pc, t2, 1.0 / 40320.0);               //  1/8!
    pc = fma(pc, t2, -1.0 / 720.0);                // -1/6!
    pc = fma(pc, t2, 1.0 / 24.0);                  //  1/4!
    pc = fma(pc, t2, -0.5);                        // -1/2!
    const double cr = fma(t2, pc, 1.0);
    const int k = (int)q & 3;                      // angle = k quarter turns + t
    const double ss = (k & 1) ? cr : sr, cc = (k & 1) ? sr : cr;
    *s = (k & 2) ? -ss : ss;
    *c = ((k + 1) & 2) ? -cc : cc;
  }
}

template <bool ROT, bool TIDAL, bool MIXED, bool EXPL>
__global__ __launch_bounds__(kWBlock) void waveform_kernel(WaveformArgs a) {
  constexpr uint32_t flags = (TIDAL ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u);
  __shared__ EventC ec;
  __shared__ WaveSite ws[kMaxSites];
  __shared__ int32_t ok;
  const int64_t e = a.base + blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  if (tid == 0) {
    double p[kNparIn];
    load_event(a, e, TIDAL, p);
    event_setup_grid(p, a.fmin, a.fmax, a.npts, a.goff, a.gf, e, flags | a.ecc_flag, ec);
    // the event's columns [b, b + npts) must lie inside a row of h
    const int64_t b = a.offsets[e];
    const bool range_ok = b >= 0 && b <= a.total - (int64_t)a.npts[e];
    int32_t st = ec.status;
    if (!range_ok) st |= kEvInvalid;
    ok = st == 0;
    if (a.status) a.status[e] = st;
  }
  __syncthreads();
  if (!ok) return;
  if (tid < n_site) {
    double p[kNparIn];
    load_event(a, e, TIDAL, p);
    SiteC sc;
    site_setup(p, a.net.site[tid], ec, sc);
    WaveSite& w = ws[tid];
    w.cdl = sc.cdl; w.sdl = sc.sdl;
    w.k1 = sc.k1; w.k0 = sc.k0;
    double pc[4][5], ptc[4][5];
    pattern_trig(sc.ct, sc.st, sc.sl, sc.cl, pc, ptc);
    for (int j = 0; j < 2; ++j)
      for (int m = 0; m < 5; ++m) {
        double fp = 0.0, fx = 0.0;
        for (int i = 0; i < 4; ++i) {
          fp = fma(sc.arm_alpha[j][i], pc[i][m], fp);
          fx = fma(sc.arm_beta[j][i], pc[i][m], fx);
        }
        w.m[j][0][m] = ec.cplus * fp;
        w.m[j][1][m] = ec.ccross * fx;
      }
    w.n_arm = sc.n_arm;
  }
  __syncthreads();

  const double tc = a.tc_s ? a.tc_s[e] : 0.0;
  const int64_t base = a.offsets[e];
  const double amp0 = exp(ec.lnA);
  double2* __restrict__ out = reinterpret_cast<double2*>(a.h) + base;
  const int64_t row = a.total;
  for (int k = tid; k < ec.n; k += kWBlock) {
    // explicit grids: ln v = (ln(pi M) + ln f)/3 from the given frequency
    const double L = EXPL ? (ec.lnpiM + log(ec.fx[k])) / 3.0 : fma((double)k, ec.dlnv, ec.lnv0);
    const double v = exp(L);
    const double iv = recip(v);
    const double iv2 = iv * iv, iv5 = iv2 * iv2 * iv;
    VPow pw;
    vpow(v, L, pw);
    const double v2 = pw.p2;
    const double f = EXPL ? ec.fx[k] : v2 * v * ec.inv_piM;
    // A(f) = A0 v^-7/2; mixed form: 2^y, y = -3.5 log2 v, with the integer
    // part of y split off exactly before the FP32 exponential
    double amp;
    if (MIXED) {
      const double y = (-3.5 / kLn2) * L, n = rint(y);
      amp = amp0 * (double)ldexpf(exp2f((float)(y - n)), (int)n);
    } else {
      amp = amp0 * iv2 * iv * sqrt(iv);
    }
    double cth, sth;
    {
      const double th = ROT ? ec.thc + eval_tau(ec.ts[kTsTheta], pw, iv5 * iv2 * iv, iv2) : ec.thc;
      // FP64 in both forms: the hour angle also sets the arrival-time phase
      // 2 pi f Delta (tens of cycles at kHz), which an FP32 cos H would move
      // by ~1e-5 rad
      sincos_moderate(th, &sth, &cth);
    }
    // cycles: Psi_PN/(2 pi) + f tc - (Phic + pi/4)/(2 pi), each reduced
    // modulo one.  f tc - n with n the integer nearest to the rounded product
    // is formed by one fused multiply-add from the exact product, so the
    // reduced fraction carries a single rounding however large f tc is.
    double pnc = eval_phase(ec.cyc, pw, iv5);
    if (ec.ecc) pnc = fma(ec.ecc_cyc, iv5 * exp((19.0 / 3.0) * (ec.ecc_lnvr - L)), pnc);
    const double pn = frac_center(pnc);
    const double ftr = fma(f, tc, -rint(f * tc));
    const double cyc = frac_center(pn + ftr + ec.cyc0);
    double2* o = out + k;
    for (int s = 0; s < n_site; ++s) {
      asm volatile("" ::: "memory");   // site constants stay in LDS rather than occupying registers
      const WaveSite& w = ws[s];
      const double cH = cth * w.cdl - sth * w.sdl;
      const double sH = sth * w.cdl + cth * w.sdl;
      const double c2H = fma(cH, cH, -sH * sH), s2H = 2.0 * (sH * cH);
      double sn, cs;
      sincos_cycles<MIXED>(frac_center(fma(f, fma(w.k1, cH, w.k0), cyc)), &sn, &cs);
      const double ca = amp * cs, sa = amp * sn;
      const double qr0 = trig5(w.m[0][0], cH, sH, c2H, s2H), qi0 = trig5(w.m[0][1], cH, sH, c2H, s2H);
      const double2 h0 = make_double2(qr0 * ca - qi0 * sa, qr0 * sa + qi0 * ca);
      *o = h0;
      o += row;
      if (w.n_arm == 3) {                 // closed triangle: third arm = -(first + second)
        const double qr1 = trig5(w.m[1][0], cH, sH, c2H, s2H), qi1 = trig5(w.m[1][1], cH, sH, c2H, s2H);
        const double2 h1 = make_double2(qr1 * ca - qi1 * sa, qr1 * sa + qi1 * ca);
        o[0] = h1;
        o[row] = make_double2(-(h0.x + h1.x), -(h0.y + h1.y));
        o += 2 * row;
      }
    }
  }
}

// The strain's derivatives with respect to the P parameters, in the rows and
// units of the Fisher matrix (whose entries are 4 Re sum w d_a h d_b h^* / S_n):
//   d_a h_i = A exp(2 pi i cyc_i) D_a,i,
// D the phase-free derivative vector of the Fisher kernels for (Mc, eta, dL,
// theta, phi, iota, psi, tc) and i Q c_a for the phase-only parameters
// (Phic, chi1z, chi2z[, Lambda1, Lambda2][, e0]); the phase in cycles exactly as
// for the strain.  Each arm of a triangle is projected with its own pattern
// map.  One workgroup per event, lanes over grid points; row (a, i) of dh
// holds parameter a at interferometer i, consecutive lanes on consecutive
// complex values.  FP64 only.
template <bool ROT, int NPI, bool EXPL>
__global__ __launch_bounds__(kWBlock) void waveform_deriv_kernel(WaveformArgs a) {
  using PO = PhaseOnly<NPI>;
  constexpr int P = PO::P;
  constexpr bool TIDAL = PO::tidal;
  constexpr uint32_t flags = (TIDAL ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u) | (PO::ecc ? kFlagEcc : 0u);
  __shared__ EventC ec;
  __shared__ SiteC sc[kMaxSites];
  __shared__ int32_t ok;
  const int64_t e = a.base + blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  if (tid == 0) {
    double p[kNparIn];
    load_event(a, e, TIDAL, p);
    event_setup_grid(p, a.fmin, a.fmax, a.npts, a.goff, a.gf, e, flags, ec);
    const int64_t b = a.offsets[e];
    const bool range_ok = b >= 0 && b <= a.total - (int64_t)a.npts[e];
    int32_t st = ec.status;
    if (!range_ok) st |= kEvInvalid;
    ok = st == 0;
    if (a.status) a.status[e] = st;
  }
  __syncthreads();
  if (!ok) return;
  if (tid < n_site) {
    double p[kNparIn];
    load_event(a, e, TIDAL, p);
    site_setup(p, a.net.site[tid], ec, sc[tid]);
  }
  __syncthreads();

  const uint32_t pm = event_rows(a.par_mask, e);
  const double tc = a.tc_s ? a.tc_s[e] : 0.0;
  const double amp0 = exp(ec.lnA);
  const AmpFactors am = amp_factors(ec);
  double2* __restrict__ out = reinterpret_cast<double2*>(a.dh) + a.offsets[e];
  const int64_t row = a.total;
  const int64_t prow = (int64_t)a.net.n_ifo * row;     // one parameter's block of rows
  for (int k = tid; k < ec.n; k += kWBlock) {
    // the event and site constants are re-read from LDS (uniform broadcast
    // reads) rather than held in registers across iterations
    asm volatile("" ::: "memory");
    Point q;
    point_setup<true, EXPL, PO::ecc>(ec, k, true, ROT, q, kPsdNone);
    VPow pw;
    vpow(q.v, q.L, pw);
    const double iv = q.iv, iv2 = iv * iv, iv5 = iv2 * iv2 * iv;
    const double amp = amp0 * iv2 * iv * sqrt(iv);
    double pnc = eval_phase(ec.cyc, pw, iv5);
    if (PO::ecc) pnc = fma(ec.ecc_cyc, q.ecv, pnc);
    const double pn = frac_center(pnc);
    const double ftr = fma(q.f, tc, -rint(q.f * tc));
    const double cyc = frac_center(pn + ftr + ec.cyc0);
    double cph[NPI];
    phase_only_coefficients<NPI>(ec, q, cph);
    double2* o = out + k;
    for (int s = 0; s < n_site; ++s) {
      asm volatile("" ::: "memory");
      const SiteC& st = sc[s];
      SitePoint sp;
      site_point<false, true>(st, q, true, sp);
      const SitePhase ph = site_phase(q, sp);
      const double cH = q.cth * st.cdl - q.sth * st.sdl;
      double sn, cs;
      sincos_cycles<false>(frac_center(fma(q.f, fma(st.k1, cH, st.k0), cyc)), &sn, &cs);
      const double ca = amp * cs, sa = amp * sn;
      for (int j = 0; j < st.n_arm; ++j) {
        const double Fp = dot4(st.arm_alpha[j], sp.P), Fx = dot4(st.arm_beta[j], sp.P);
        double Dr[P], Di[P];
        derivative_vector(am, q, ph, Fp, Fx, dot4(st.arm_alpha[j], sp.PH), dot4(st.arm_beta[j], sp.PH),
                          dot4(st.arm_alpha[j], sp.Pt), dot4(st.arm_beta[j], sp.Pt), Dr, Di);
        const double Qr = am.cplus * Fp, Qi = am.ccross * Fx;
#pragma unroll
        for (int i = 0; i < NPI; ++i) {          // i Q c
          Dr[8 + i] = -Qi * cph[i];
          Di[8 + i] = Qr * cph[i];
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
          const bool in = (pm >> r) & 1u;
          o[r * prow] = in ? make_double2(Dr[r] * ca - Di[r] * sa, Dr[r] * sa + Di[r] * ca)
                           : make_double2(0.0, 0.0);
        }
        o += row;
      }
    }
  }
}

}  // namespace

template <bool MIXED, bool EXPL>
void launch_waveform_t(const WaveformArgs& a, bool tidal, bool rot, dim3 grid, dim3 block,
                       hipStream_t stream) {
  if (tidal && rot) hipLaunchKernelGGL((waveform_kernel<true, true, MIXED, EXPL>), grid, block, 0, stream, a);
  else if (tidal) hipLaunchKernelGGL((waveform_kernel<false, true, MIXED, EXPL>), grid, block, 0, stream, a);
  else if (rot) hipLaunchKernelGGL((waveform_kernel<true, false, MIXED, EXPL>), grid, block, 0, stream, a);
  else hipLaunchKernelGGL((waveform_kernel<false, false, MIXED, EXPL>), grid, block, 0, stream, a);
}

// An explicit grid (a.gf set) selects the instantiations that read it.
hipError_t launch_waveform(const WaveformArgs& a0, bool tidal, bool rot, bool mixed, hipStream_t stream) {
  return launch_slices(a0, a0.n, 1, kWBlock, [&](const WaveformArgs& a, dim3 grid, dim3 block) {
    if (a.gf) {
      if (mixed) launch_waveform_t<true, true>(a, tidal, rot, grid, block, stream);
      else launch_waveform_t<false, true>(a, tidal, rot, grid, block, stream);
    } else {
      if (mixed) launch_waveform_t<true, false>(a, tidal, rot, grid, block, stream);
      else launch_waveform_t<false, false>(a, tidal, rot, grid, block, stream);
    }
  });
}

template <int NPI, bool EXPL>
void launch_deriv_n(const WaveformArgs& a, bool rot, dim3 grid, dim3 block, hipStream_t stream) {
  if (rot) hipLaunchKernelGGL((waveform_deriv_kernel<true, NPI, EXPL>), grid, block, 0, stream, a);
  else hipLaunchKernelGGL((waveform_deriv_kernel<false, NPI, EXPL>), grid, block, 0, stream, a);
}

template <bool EXPL>
void launch_deriv_t(const WaveformArgs& a, int npi, bool rot, dim3 grid, dim3 block, hipStream_t stream) {
  switch (npi) {
    case 6: launch_deriv_n<6, EXPL>(a, rot, grid, block, stream); break;
    case 5: launch_deriv_n<5, EXPL>(a, rot, grid, block, stream); break;
    case 4: launch_deriv_n<4, EXPL>(a, rot, grid, block, stream); break;
    default: launch_deriv_n<3, EXPL>(a, rot, grid, block, stream);
  }
}

hipError_t launch_waveform_deriv(const WaveformArgs& a0, int npi, bool rot, hipStream_t stream) {
  return launch_slices(a0, a0.n, 1, kWBlock, [&](const WaveformArgs& a, dim3 grid, dim3 block) {
    if (a.gf) launch_deriv_t<true>(a, npi, rot, grid, block, stream);
    else launch_deriv_t<false>(a, npi, rot, grid, block, stream);
  });
}

}  // namespace gwf

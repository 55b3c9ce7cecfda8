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
#include "gwf_waveform.hpp"

namespace gwf {

namespace {

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

}  // namespace gwf

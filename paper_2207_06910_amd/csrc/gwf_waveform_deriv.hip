// gwf_waveform_deriv.hip -- the strain's derivatives with respect to the
// Fisher parameters at every interferometer and grid point (the d h / d theta
// arrays the paper's Fisher matrices are built from, sec. 3.2), phase in
// cycles as for the strain (gwf_waveform.hip).
#include "gwf_waveform.hpp"

namespace gwf {

namespace {

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

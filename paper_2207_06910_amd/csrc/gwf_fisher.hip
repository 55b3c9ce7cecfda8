// gwf_fisher.hip -- SNR and Fisher-matrix kernels (plain FP64 form).
//
// One workgroup of 256 lanes per event.  The workgroup first builds the
// event's constants (PN-series coefficients, grid, amplitude) and each
// site's constants (pattern maps, delay and PSD factors) in LDS; every lane
// then walks the event's frequency grid with stride 256, evaluates the
// derivative vectors of all interferometers at its frequency in registers
// and accumulates the noise-weighted Gram matrix; a fixed-order wavefront +
// LDS reduction produces the event's matrix.  Nothing is atomically added,
// so results are bitwise reproducible.
//
// The accumulation itself (gwf_fisher_body.hpp) is shared with the batched
// work-item form (gwf_batched.hip).
//
// Gram structure exploited (exact algebra, no approximation): the derivative
// vectors with respect to Phic, chi1, chi2, Lambda1, Lambda2 are i Q c_a(f)
// with the same real c_a(f) for every interferometer, so their blocks follow
// from per-frequency network sums W = sum_i w_i |Q_i|^2 and
// U_b = sum_i w_i Re(i Q_i D_b,i^*):
//   Gamma_ab += W c_a c_b   (a, b phase-only),   Gamma_ba += U_b c_a,
// and only the 8x8 block of (Mc, eta, dL, theta, phi, iota, psi, tc) needs a
// per-interferometer rank-2 update.
#include "gwf_fisher_body.hpp"

namespace gwf {

// Declared for 2 x kBlock lanes so that the register budget is that of two
// wavefronts per SIMD (256 registers); launched with kBlock lanes, two
// workgroups (about 63 KB of LDS each: 54 KB of FisherLds, the event's
// 1.1 KB of constants and 6.9 KB for eight sites) then share a compute unit,
// which hides the latency of the LDS constant reads and of the
// transcendental sequences.
// (The P = 11 instantiation keeps the one-wavefront budget: under the
// two-wavefront cap it spills.)
static_assert(64 + kMaxSites <= kBlock, "site set-up lanes in the second wavefront");

template <int NPI_, bool ROT, bool EXPL, bool TAB>
__global__ __launch_bounds__(FisherDims<NPI_>::TIDAL ? 2 * kBlock : kBlock) void fisher_kernel(FisherArgs a) {
  using Dm = FisherDims<NPI_>;
  using PO = PhaseOnly<NPI_>;
  constexpr int P = Dm::P, NPI = Dm::NPI, NACC = Dm::NACC;
  constexpr uint32_t flags = (PO::tidal ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u) | (PO::ecc ? kFlagEcc : 0u);

  __shared__ EventC ec;
  __shared__ SiteC sc[kMaxSites];
  __shared__ FisherLds L;
  __shared__ int32_t skip, bad;

  const int64_t e = a.base + blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  double p[kNparIn];
  load_par(a.par, a.ld, e, PO::tidal, PO::ecc ? a.ecc : nullptr, a.fref, p);
  // the event's constants on lane 0 and the sites' on the second wavefront,
  // at the same time (a site needs only the parameters and pi M)
  if (tid == 0) {
    event_setup_grid(p, a.fmin, a.fmax, a.npts, a.goff, a.gf, e, flags, ec);
    int32_t sk = ec.status;
    if (!sk && a.snr_pre && !(a.snr_pre[e] > a.snr_th)) sk = kEvSkipped;
    skip = sk;
    bad = 0;
  } else if (tid >= 64 && tid < 64 + n_site) {
    const int s = tid - 64;
    site_setup(p, a.net.site[s], kPi * total_mass_s(p), sc[s],
               select_ifo(site_arms_on(a.active, a.ld, e, a.net, s), a.net, s, a.ifo_sel));
  }
  __syncthreads();
  if (skip) {
    for (int i = tid; i < P * P; i += kBlock) a.fisher[(int64_t)i * a.n + e] = 0.0;
    if (tid == 0) {
      if (!a.snr_pre && a.snr) a.snr[e] = 0.0;
      a.status[e] = skip;
    }
    return;
  }

  double t = 0.0;
  fisher_sums<NPI, ROT, false, true, EXPL, TAB>(ec, sc, n_site, 0, ec.n, L, &t);
  if (tid < NACC) {
    int r, c;
    slot_position(tid, NPI, r, c);
    if (r == 8 && c == 8 && a.snr) a.snr[e] = sqrt(t);     // Gamma_{Phic,Phic} = SNR^2
    const double v = rows_in(event_rows(a.par_mask, e), r, c) ? t : 0.0;
    if (!isfinite(v)) atomicOr(&bad, 1);
    a.fisher[((int64_t)r * P + c) * a.n + e] = v;
    a.fisher[((int64_t)c * P + r) * a.n + e] = v;
  }
  __syncthreads();
  // one launch per interferometer (ifo_sel > 1 after the first) adds its bit
  if (tid == 0) {
    const int32_t f = bad ? kEvNonFinite : 0;
    a.status[e] = a.ifo_sel > 1 ? (a.status[e] | f) : f;
  }
}

// SNR only, with the SNR of every interferometer.  Same grid, weights and
// patterns as the Fisher kernel; no derivatives.
template <bool ROT, bool EXPL>
__global__ __launch_bounds__(kBlock) void snr_kernel(SnrArgs a) {
  constexpr uint32_t flags = ROT ? kFlagRot : 0u;
  __shared__ EventC ec;
  __shared__ SiteC sc[kMaxSites];
  __shared__ double red[kWaves][kMaxIfo + 1];
  const int64_t e = a.base + blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  double p[kNparIn];
  load_par(a.par, a.ld, e, a.tidal, nullptr, nullptr, p);
  // the event's constants on lane 0 and the sites' on the second wavefront, at once
  if (tid == 0)
    event_setup_grid(p, a.fmin, a.fmax, a.npts, a.goff, a.gf, e, flags | (a.tidal ? kFlagTidal : 0u), ec);
  else if (tid >= 64 && tid < 64 + n_site)
    site_setup(p, a.net.site[tid - 64], kPi * total_mass_s(p), sc[tid - 64]);
  __syncthreads();
  if (ec.status) {
    if (tid == 0) {
      a.snr[e] = 0.0;
      if (a.status) a.status[e] = ec.status;
    }
    if (a.snr_ifo)
      for (int i = tid; i < a.net.n_ifo; i += kBlock) a.snr_ifo[(int64_t)i * a.n + e] = 0.0;
    return;
  }
  // slot 3 s + k holds arm k of site s
  double acc[3 * kMaxSites];
#pragma unroll
  for (int i = 0; i < 3 * kMaxSites; ++i) acc[i] = 0.0;
  const double cplus = ec.cplus, ccross = ec.ccross;
  for (int k = tid; k < ec.n; k += kBlock) {
    __asm__ volatile("" ::: "memory");
    Point q;
    point_setup<false, EXPL>(ec, k, false, ROT, q);
#pragma unroll
    for (int s = 0; s < kMaxSites; ++s) {
      if (s < n_site) {
        const SiteC& st = sc[s];
        SitePoint sp;
        site_point<false, false>(st, q, false, sp);
        if (st.n_arm == 3) {
          const double p0 = cplus * dot4(st.arm_alpha[0], sp.P), x0 = ccross * dot4(st.arm_beta[0], sp.P);
          const double p1 = cplus * dot4(st.arm_alpha[1], sp.P), x1 = ccross * dot4(st.arm_beta[1], sp.P);
          const double p2 = -(p0 + p1), x2 = -(x0 + x1);
          acc[3 * s] = fma(sp.om, fma(p0, p0, x0 * x0), acc[3 * s]);
          acc[3 * s + 1] = fma(sp.om, fma(p1, p1, x1 * x1), acc[3 * s + 1]);
          acc[3 * s + 2] = fma(sp.om, fma(p2, p2, x2 * x2), acc[3 * s + 2]);
        } else {
          const double p0 = cplus * dot4(st.arm_alpha[0], sp.P), x0 = ccross * dot4(st.arm_beta[0], sp.P);
          acc[3 * s] = fma(sp.om, fma(p0, p0, x0 * x0), acc[3 * s]);
        }
      }
    }
  }
  const int wave = tid >> 6, lane = tid & 63;
  int ifo = 0;
#pragma unroll
  for (int s = 0; s < kMaxSites; ++s) {
    if (s < n_site) {
      const int na = sc[s].n_arm;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        if (k < na) {
          const double t = wave_sum(acc[3 * s + k]);
          if (lane == 0) red[wave][ifo] = t;
          ++ifo;
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    bool bad = false;
    for (int i = 0; i < a.net.n_ifo; ++i) {
      double t = red[0][i];
      for (int w = 1; w < kWaves; ++w) t += red[w][i];
      if (a.active && !a.active[(int64_t)i * a.ld + e]) t = 0.0;   // off for this event
      tot += t;
      if (a.snr_ifo) a.snr_ifo[(int64_t)i * a.n + e] = sqrt(t);
    }
    if (!isfinite(tot)) bad = true;
    a.snr[e] = sqrt(tot);
    if (a.status) a.status[e] = bad ? kEvNonFinite : 0;
  }
}

template <int NPI, bool EXPL>
void launch_fisher_n(const FisherArgs& a, bool rot, dim3 grid, dim3 block, hipStream_t stream) {
  const bool tab = net_has_tables(a.net);
  if (rot && tab) hipLaunchKernelGGL((fisher_kernel<NPI, true, EXPL, true>), grid, block, 0, stream, a);
  else if (rot) hipLaunchKernelGGL((fisher_kernel<NPI, true, EXPL, false>), grid, block, 0, stream, a);
  else if (tab) hipLaunchKernelGGL((fisher_kernel<NPI, false, EXPL, true>), grid, block, 0, stream, a);
  else hipLaunchKernelGGL((fisher_kernel<NPI, false, EXPL, false>), grid, block, 0, stream, a);
}

template <bool EXPL>
void launch_fisher_t(const FisherArgs& a, int npi, bool rot, dim3 grid, dim3 block, hipStream_t stream) {
  switch (npi) {
    case 6: launch_fisher_n<6, EXPL>(a, rot, grid, block, stream); break;
    case 5: launch_fisher_n<5, EXPL>(a, rot, grid, block, stream); break;
    case 4: launch_fisher_n<4, EXPL>(a, rot, grid, block, stream); break;
    default: launch_fisher_n<3, EXPL>(a, rot, grid, block, stream);
  }
}

// An explicit grid (a.gf set) selects the instantiations that read it.
hipError_t launch_fisher(const FisherArgs& a0, int npi, bool rot, hipStream_t stream) {
  return launch_slices(a0, a0.n, 1, kBlock, [&](const FisherArgs& a, dim3 grid, dim3 block) {
    if (a.gf) launch_fisher_t<true>(a, npi, rot, grid, block, stream);
    else launch_fisher_t<false>(a, npi, rot, grid, block, stream);
  });
}

hipError_t launch_snr(const SnrArgs& a0, bool rot, hipStream_t stream) {
  return launch_slices(a0, a0.n, 1, kBlock, [&](const SnrArgs& a, dim3 grid, dim3 block) {
    if (a.gf) {
      if (rot) hipLaunchKernelGGL((snr_kernel<true, true>), grid, block, 0, stream, a);
      else hipLaunchKernelGGL((snr_kernel<false, true>), grid, block, 0, stream, a);
    } else {
      if (rot) hipLaunchKernelGGL((snr_kernel<true, false>), grid, block, 0, stream, a);
      else hipLaunchKernelGGL((snr_kernel<false, false>), grid, block, 0, stream, a);
    }
  });
}

}  // namespace gwf

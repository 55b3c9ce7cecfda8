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
// Gram structure exploited (exact algebra, no approximation): the derivative
// vectors with respect to Phic, chi1, chi2, Lambda1, Lambda2 are i Q c_a(f)
// with the same real c_a(f) for every interferometer, so their blocks follow
// from per-frequency network sums W = sum_i w_i |Q_i|^2 and
// U_b = sum_i w_i Re(i Q_i D_b,i^*):
//   Gamma_ab += W c_a c_b   (a, b phase-only),   Gamma_ba += U_b c_a,
// and only the 8x8 block of (Mc, eta, dL, theta, phi, iota, psi, tc) needs a
// per-interferometer rank-2 update.
//
// The 8x8 block (36 doubles) is accumulated in registers.  The phase-only
// blocks are a small dense contraction over frequency, X = sum_f a_f c_f^T
// with a_f = (U_0..U_7, W c_0..W c_{NPI-1}) and c_f = (c_0..c_{NPI-1}):
// every iteration each wavefront stages its 64 points' a_f and c_f in LDS
// and folds them into a 16x16 FP64 accumulator with 16 MFMA 16x16x4 steps
// (k = frequency), which keeps those 55 sums out of the lanes' registers.
#include "gwf_kernels.hpp"

namespace gwf {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kRowsA = 13;        // 8 U rows + up to 5 W c rows
constexpr int kRowsB = 5;         // up to 5 c rows
constexpr int kTileLd = 64 + 2;   // padded row stride (doubles)

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Load an event's 13 parameters (missing tidal rows read as zero).
__device__ inline void load_par(const double* __restrict__ par, int64_t ld, int64_t e, bool tidal,
                                double p[13]) {
  for (int r = 0; r < 13; ++r) p[r] = (r < 11 || tidal) ? par[r * ld + e] : 0.0;
}

}  // namespace

// Declared for 2 x kBlock lanes so that the register budget is that of two
// wavefronts per SIMD (256 registers); launched with kBlock lanes, two
// workgroups (45 KB of LDS each) then share a compute unit, which hides the
// latency of the LDS constant reads and of the transcendental sequences.
template <bool TIDAL, bool ROT>
__global__ __launch_bounds__(TIDAL ? 2 * kBlock : kBlock) void fisher_kernel(FisherArgs a) {
  constexpr int P = TIDAL ? 13 : 11;
  constexpr int NPI = P - 8;                       // phase-only parameters
  constexpr int NG = 36, NX = 8 * NPI, NY = NPI * (NPI + 1) / 2;
  constexpr int NACC = NG + NX + NY;               // SNR^2 = Gamma_{Phic,Phic}
  constexpr uint32_t flags = (TIDAL ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u);

  __shared__ EventC ec;
  __shared__ SiteC sc[kMaxSites];
  __shared__ double red[kWaves][NACC];
  __shared__ double stA[kWaves][kRowsA][kTileLd];   // staged a_f, [row][point]
  __shared__ double stB[kWaves][kRowsB][kTileLd];   // staged c_f
  __shared__ int32_t skip;

  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  double p[13];
  load_par(a.par, a.ld, e, TIDAL, p);
  if (tid == 0) {
    event_setup(p, a.fmin[e], a.fmax ? a.fmax[e] : 0.0, a.npts[e], flags, ec);
    int32_t sk = ec.status;
    if (!sk && a.snr_pre && !(a.snr_pre[e] > a.snr_th)) sk = kEvSkipped;
    skip = sk;
  }
  __syncthreads();
  if (skip) {
    for (int i = tid; i < P * P; i += kBlock) a.fisher[(int64_t)i * a.n + e] = 0.0;
    if (tid == 0) {
      if (!a.snr_pre) a.snr[e] = 0.0;
      a.status[e] = skip;
    }
    return;
  }
  if (tid < n_site) site_setup(p, a.net.site[tid], ec, sc[tid]);
  __syncthreads();

  double G[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) G[i] = 0.0;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  const int wave = tid >> 6, lane = tid & 63;
  const int mrow = lane & 15, mk = lane >> 4;      // MFMA operand position of this lane
  double(*A)[kTileLd] = stA[wave];
  double(*B)[kTileLd] = stB[wave];

  const int n = ec.n;
  const int iters = (n + kBlock - 1) / kBlock;    // same trip count for every lane
  for (int it = 0; it < iters; ++it) {
    // The per-event constants stay in LDS and are re-read every iteration
    // (uniform broadcast reads); hoisting them out of the loop would need
    // more registers than a lane has.
    __asm__ volatile("" ::: "memory");
    const int k = it * kBlock + tid;
    double U[8], W = 0.0, cph[NPI];
#pragma unroll
    for (int b = 0; b < 8; ++b) U[b] = 0.0;
#pragma unroll
    for (int i = 0; i < NPI; ++i) cph[i] = 0.0;
    if (k < n) accumulate_point<TIDAL, ROT>(ec, sc, n_site, k, G, U, W, cph);
    // stage this point's row (points past the grid end contribute zeros)
#pragma unroll
    for (int b = 0; b < 8; ++b) A[b][lane] = U[b];
#pragma unroll
    for (int i = 0; i < NPI; ++i) {
      A[8 + i][lane] = W * cph[i];
      B[i][lane] = cph[i];
    }
    __builtin_amdgcn_wave_barrier();
    // X += A^T B over this wavefront's 64 points: k-step s takes points 16 mk + s
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
      const double av = mrow < 8 + NPI ? A[mrow][16 * mk + s2] : 0.0;
      const double bv = mrow < NPI ? B[mrow][16 * mk + s2] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
  }

  // ---- deterministic reduction: wavefront butterflies, then the 4 waves in order
#pragma unroll
  for (int i = 0; i < NG; ++i) { double t = wave_sum(G[i]); if (lane == 0) red[wave][i] = t; }
  // register r of lane (mk, mrow) holds accumulator element (4 r + mk, mrow):
  // rows 0..7 are the U_b rows (cols 0..NPI-1), rows 8..8+NPI-1 the W c_i
  // rows (upper triangle kept)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * r + mk, col = mrow;
    int slot = -1;
    if (row < 8 && col < NPI) slot = NG + row * NPI + col;
    else if (row >= 8 && row < 8 + NPI && col >= row - 8 && col < NPI) {
      const int i = row - 8;
      slot = NG + NX + i * NPI - (i * (i - 1)) / 2 + (col - i);
    }
    if (slot >= 0) red[wave][slot] = acc[r];
  }
  __syncthreads();
  __shared__ int32_t bad;
  if (tid == 0) bad = 0;
  __syncthreads();
  if (tid < NACC) {
    double t = red[0][tid];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t += red[w][tid];
    if (!isfinite(t)) atomicOr(&bad, 1);
    int r, c;
    slot_position(tid, NPI, r, c);
    if (r == 8 && c == 8) a.snr[e] = sqrt(t);     // Gamma_{Phic,Phic} = SNR^2
    {
      a.fisher[((int64_t)r * P + c) * a.n + e] = t;
      a.fisher[((int64_t)c * P + r) * a.n + e] = t;
    }
  }
  __syncthreads();
  if (tid == 0) a.status[e] = bad ? kEvNonFinite : 0;
}

// SNR only, with the SNR of every interferometer.  Same grid, weights and
// patterns as the Fisher kernel; no derivatives.
template <bool ROT>
__global__ __launch_bounds__(kBlock) void snr_kernel(SnrArgs a) {
  constexpr uint32_t flags = ROT ? kFlagRot : 0u;
  __shared__ EventC ec;
  __shared__ SiteC sc[kMaxSites];
  __shared__ double red[kWaves][kMaxIfo + 1];
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  double p[13];
  load_par(a.par, a.ld, e, a.tidal, p);
  if (tid == 0) event_setup(p, a.fmin[e], a.fmax ? a.fmax[e] : 0.0, a.npts[e], flags | (a.tidal ? kFlagTidal : 0u), ec);
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
  if (tid < n_site) site_setup(p, a.net.site[tid], ec, sc[tid]);
  __syncthreads();
  // slot 3 s + k holds arm k of site s
  double acc[3 * kMaxSites];
#pragma unroll
  for (int i = 0; i < 3 * kMaxSites; ++i) acc[i] = 0.0;
  const double cplus = ec.cplus, ccross = ec.ccross;
  for (int k = tid; k < ec.n; k += kBlock) {
    __asm__ volatile("" ::: "memory");
    Point q;
    point_setup(ec, k, false, ROT, q);
#pragma unroll
    for (int s = 0; s < kMaxSites; ++s) {
      if (s < n_site) {
        const SiteC& st = sc[s];
        SitePoint sp;
        site_point(st, q, false, sp);
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
      tot += t;
      if (a.snr_ifo) a.snr_ifo[(int64_t)i * a.n + e] = sqrt(t);
    }
    if (!isfinite(tot)) bad = true;
    a.snr[e] = sqrt(tot);
    if (a.status) a.status[e] = bad ? kEvNonFinite : 0;
  }
}

hipError_t launch_fisher(const FisherArgs& a, bool tidal, bool rot, hipStream_t stream) {
  dim3 grid((unsigned)a.n), block(kBlock);
  if (tidal && rot) hipLaunchKernelGGL((fisher_kernel<true, true>), grid, block, 0, stream, a);
  else if (tidal) hipLaunchKernelGGL((fisher_kernel<true, false>), grid, block, 0, stream, a);
  else if (rot) hipLaunchKernelGGL((fisher_kernel<false, true>), grid, block, 0, stream, a);
  else hipLaunchKernelGGL((fisher_kernel<false, false>), grid, block, 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_snr(const SnrArgs& a, bool rot, hipStream_t stream) {
  dim3 grid((unsigned)a.n), block(kBlock);
  if (rot) hipLaunchKernelGGL((snr_kernel<true>), grid, block, 0, stream, a);
  else hipLaunchKernelGGL((snr_kernel<false>), grid, block, 0, stream, a);
  return hipGetLastError();
}

}  // namespace gwf

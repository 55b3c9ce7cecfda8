// gwf_adjoint.hip -- the adjoint (backward) pass of the Fisher/SNR map with
// respect to the detector parameters; the per-point mathematics and its
// derivation are in gwf_adjoint.hpp.
//
//   adjoint_kernel  one workgroup of 128 lanes per event: the event's
//                   constants, the contractions of its symmetrised Gbar
//                   (AdjEventC) and the sites' constants (SiteC, AdjSiteC)
//                   in LDS; every lane walks the grid with a stride of the
//                   workgroup size, forms the point quantities once, and
//                   each pair of lanes adds its two points' contributions per
//                   site to one LDS column (one LDS add per value; every
//                   address has one writer, so the sums are in program
//                   order); the columns are reduced in
//                   a fixed order and combined into the event's gradient
//                   terms.
//   reduce_kernel   one workgroup per output component sums the events'
//                   terms in a fixed order, so the gradient is bitwise
//                   reproducible.
//
// The batched form (gwf_plan_adjoint) runs the same per-point mathematics
// over a plan's work items:
//   adj_setup_kernel        one lane per event (AdjEventC from Gbar) and one
//                   per (event, site) (AdjSiteC), into the plan's adjoint
//                   workspace (the plan's set-up kernel has written EventC
//                   and SiteC);
//   adjoint_items_kernel    one workgroup of 128 lanes per work item (event,
//                   point range), in the plan's longest-first order; the
//                   event's and sites' constants are read through the
//                   constant address space (scalar loads into SGPRs); the
//                   item's per-site sums go to its slot (deterministic:
//                   fixed reduction order, slots in event order);
//   adjoint_combine_kernel  one lane per event sums its items' slots in item
//                   order and forms the event's gradient terms; the
//                   reduce_kernel then sums the events.
#include "gwf_adjoint.hpp"
#include "gwf_batched.hpp"
#include "gwf_kernels.hpp"

namespace gwf {

namespace {

constexpr int kABlock = 128;          // lanes of a workgroup (both forms)
constexpr int kSlots = kAdjN;         // LDS accumulator values per site and column
// The grid walk's stride and anchor spacing (points): they fix the grid values
// at every point, whatever the workgroup size.
constexpr int kWalk = 128;
constexpr int kAnchor = 16 * kWalk;

__device__ inline double wave_sum_a(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// The sums of points [k0, k1) of one event into LDS columns (zeroed by the
// caller, one writer per address, so the sums are in program order), by a
// workgroup of nb lanes (a multiple of kWalk dividing kAnchor; k0 a multiple
// of kWalk): lane t takes the points k0 + t, k0 + t + nb, ...
// PAIR = false, one column per lane, accl[(s kSlots + i) nb + lane];
// PAIR = true, each pair of lanes adds its two points' values and the even
// lane adds that to column lane / 2 of nb / 2, which halves the LDS a
// workgroup needs for 3 VALU instructions per value.
//
// Grid values: v, 1/v and v^-12.42 at point k are evaluated directly at
// a + k mod kWalk, a = the multiple of kAnchor at or below k, and carried
// from there by (k - a) / kWalk multiplications by the exact ratio over
// kWalk points, in that order.  The sum of Gbar-weighted terms cancels
// strongly when Gbar is an ill-conditioned covariance, so these values must
// not depend on where a work item starts or on the workgroup size: every
// form (batched, per event, any nb) sees the same values at every point.
template <int NPI, bool ROT, bool TAB, bool PAIR>
__device__ __attribute__((always_inline)) inline void adjoint_sums(const EventC& ec, const AdjEventC& ae,
                                                                   const SiteC* sc, const AdjSiteC* as, int n_site,
                                                                   int k0, int k1, int nb, double* accl) {
  const int tid = threadIdx.x;
  const int r = tid % kWalk;             // k mod kWalk at every point of the lane
  int k = k0 + tid;
  int a = k - k % kAnchor;
  GridWalk gw;
  gw.start(ec, a + r, kWalk);
  for (int q = (k - a) / kWalk; q > 0; --q) gw.step();
  const int iters = (k1 - k0 + nb - 1) / nb;
  for (int it = 0; it < iters; ++it, k += nb) {
    asm volatile("" ::: "memory");   // constants are re-read rather than held in registers
    if (it > 0) {
      if (k - a >= kAnchor) {          // the lane's point has passed an anchor
        a = k - k % kAnchor;
        gw.anchor(ec, a + r);
        for (int q = (k - a) / kWalk; q > 0; --q) gw.step();
      } else {
        for (int q = nb / kWalk; q > 0; --q) gw.step();
      }
    }
    const bool in = k < k1;
    if (PAIR) {                      // both lanes of a pair take part in each exchange
      const int cols = nb >> 1;
      AdjPoint ap;
      if (in) adjoint_point_setup<NPI, ROT>(ec, ae, k, ap, gw.val);
      for (int s = 0; s < n_site; ++s) {
        asm volatile("" ::: "memory");
        double acc[kAdjN];
#pragma unroll
        for (int i = 0; i < kAdjN; ++i) acc[i] = 0.0;
        if (in) adjoint_site<TAB>(ae, sc[s], as[s], ap, acc);
#pragma unroll
        for (int i = 0; i < kSlots; ++i) {
          const double v = acc[i] + __shfl_xor(acc[i], 1, 64);
          if ((tid & 1) == 0) atomicAdd(&accl[(s * kSlots + i) * cols + (tid >> 1)], v);
        }
      }
    } else if (in) {
      AdjPoint ap;
      adjoint_point_setup<NPI, ROT>(ec, ae, k, ap, gw.val);
      for (int s = 0; s < n_site; ++s) {
        asm volatile("" ::: "memory");
        double acc[kAdjN];
#pragma unroll
        for (int i = 0; i < kAdjN; ++i) acc[i] = 0.0;
        adjoint_site<TAB>(ae, sc[s], as[s], ap, acc);
#pragma unroll
        for (int i = 0; i < kSlots; ++i) atomicAdd(&accl[(s * kSlots + i) * nb + tid], acc[i]);
      }
    }
  }
}

// adjoint_sums with PAIR = false and two grid points per lane and iteration,
// k and k + nb (the same walk, taken two points at a time): the two points'
// site terms are independent instruction streams the compiler interleaves,
// and each site's constants are read once for both.  A point past k1 is
// evaluated as the item's last point with zero weight (every term of
// adjoint_site carries the weight), so the site code has no branch; its walk
// values would overflow on a short grid.  The column gets the two points'
// sum per site and iteration.
template <int NPI, bool ROT, bool TAB>
__device__ __attribute__((always_inline)) inline void adjoint_sums2(const EventC& ec, const AdjEventC& ae,
                                                                    const SiteC* sc, const AdjSiteC* as, int n_site,
                                                                    int k0, int k1, int nb, double* accl) {
  const int tid = threadIdx.x;
  const int r = tid % kWalk;
  int k = k0 + tid;
  int a = k - k % kAnchor;
  GridWalk gw;
  gw.start(ec, a + r, kWalk);
  for (int q = (k - a) / kWalk; q > 0; --q) gw.step();
  // from the lane's current point to kn = that point + nb
  auto advance = [&](int kn) {
    if (kn - a >= kAnchor) {
      a = kn - kn % kAnchor;
      gw.anchor(ec, a + r);
      for (int q = (kn - a) / kWalk; q > 0; --q) gw.step();
    } else {
      for (int q = nb / kWalk; q > 0; --q) gw.step();
    }
  };
  const int iters = (k1 - k0 + 2 * nb - 1) / (2 * nb);
  for (int it = 0; it < iters; ++it, k += 2 * nb) {
    asm volatile("" ::: "memory");   // constants are re-read rather than held in registers
    // grid values of point kk, or of the item's last point where kk >= k1
    auto values = [&](int kk, double* vv) {
      if (kk < k1) {
#pragma unroll
        for (int i = 0; i < 3; ++i) vv[i] = gw.val[i];
      } else {
        const double L = fma((double)(k1 - 1), ec.dlnv, ec.lnv0);
        vv[0] = exp(L);
        vv[1] = exp(-L);
        vv[2] = exp(-12.42 * L);
      }
    };
    if (it > 0) advance(k);
    AdjPoint p1, p2;
    double v1[3], v2[3];
    values(k, v1);
    adjoint_point_setup<NPI, ROT>(ec, ae, k < k1 ? k : k1 - 1, p1, v1);
    advance(k + nb);
    values(k + nb, v2);
    adjoint_point_setup<NPI, ROT>(ec, ae, k + nb < k1 ? k + nb : k1 - 1, p2, v2);
    if (k >= k1) p1.q.w4A2 = 0.0;
    if (k + nb >= k1) p2.q.w4A2 = 0.0;
    for (int s = 0; s < n_site; ++s) {
      asm volatile("" ::: "memory");
      double acc[kAdjN];
#pragma unroll
      for (int i = 0; i < kAdjN; ++i) acc[i] = 0.0;
      adjoint_site<TAB>(ae, sc[s], as[s], p1, acc);
      adjoint_site<TAB>(ae, sc[s], as[s], p2, acc);
#pragma unroll
      for (int i = 0; i < kSlots; ++i) atomicAdd(&accl[(s * kSlots + i) * nb + tid], acc[i]);
    }
  }
}

// The site sums of the workgroup's columns (as adjoint_sums left them), in a
// fixed order: wave w of the nb / 64 takes the values t = w, w + nb / 64, ...;
// each lane adds its columns in column order, then the wavefront butterfly.
template <bool PAIR>
__device__ inline void adjoint_columns(const double* accl, int width, int nb, double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cols = PAIR ? nb >> 1 : nb;
  for (int t = wave; t < width; t += nb >> 6) {
    double c = 0.0;
    for (int j = lane; j < cols; j += 64) c += accl[t * cols + j];
    const double v = wave_sum_a(c);
    if (lane == 0) out[t] = v;
  }
}

// Gbar of event e from [P][P][n], symmetrised and zero outside its rows.
struct GbarOf {
  const double* g;
  int64_t n, e;
  int P;
  uint32_t pm;
  __device__ double operator()(int i, int j) const {
    return rows_in(pm, i, j) ? 0.5 * (g[(int64_t)(i * P + j) * n + e] + g[(int64_t)(j * P + i) * n + e]) : 0.0;
  }
};

struct GbarLds {
  const double* g;
  int P;
  __device__ double operator()(int i, int j) const { return g[i * P + j]; }
};

// Two wavefronts per SIMD: the registers are capped at 256 (the sums live in
// LDS, not in registers).
template <int NPI, bool ROT, bool TAB>
__global__ __launch_bounds__(kABlock, 2) void adjoint_kernel(AdjointArgs a) {
  using PO = PhaseOnly<NPI>;
  constexpr int P = PO::P;
  constexpr bool TIDAL = PO::tidal;
  constexpr uint32_t flags = (TIDAL ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u) | (PO::ecc ? kFlagEcc : 0u);
  __shared__ EventC ec;
  __shared__ AdjEventC ae;
  __shared__ SiteC sc[kMaxSites];
  __shared__ AdjSiteC as[kMaxSites];
  __shared__ double Gb[P * P];
  extern __shared__ double accl[];      // [n_site][kSlots][kABlock / 2]
  __shared__ double site_acc[kMaxSites * kSlots];
  __shared__ int32_t ok;
  const int64_t e = a.base + blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  double p[kNparIn];
  for (int r = 0; r < 13; ++r) p[r] = (r < 11 || TIDAL) ? a.par[r * a.ld + e] : 0.0;
  p[13] = PO::ecc && a.ecc ? a.ecc[e] : 0.0;
  p[14] = PO::ecc && a.fref ? a.fref[e] : 0.0;
  if (tid == 0) {
    event_setup(p, a.fmin[e], a.fmax ? a.fmax[e] : 0.0, a.npts[e], flags, ec);
    ok = ec.status == 0 && (a.status == nullptr || a.status[e] == 0);
  }
  __syncthreads();
  const uint32_t pm = event_rows(a.par_mask, e);
  for (int t = tid; t < P * P; t += kABlock) {
    const int i = t / P, j = t - i * P;
    const double g = GbarOf{a.gbar, a.n, e, P, pm}(i, j);
    Gb[t] = g;
    if (!finite(g)) ok = 0;          // every writer stores the same value
  }
  __syncthreads();
  double* ge = a.grad_event + e * (int64_t)(n_site * 4);
  if (!ok) {
    if (tid < n_site * 4) ge[tid] = 0.0;
    return;
  }
  if (tid == 0) adj_event_setup<NPI>(ec, GbarLds{Gb, P}, ae);
  if (tid < n_site) {
    const uint32_t arms = site_arms_on(a.active, a.ld, e, a.net, tid);
    site_setup(p, a.net.site[tid], ec, sc[tid], arms);
    adj_site_setup(p, a.net.site[tid], sc[tid], as[tid], arms);
  }
  for (int t = tid; t < n_site * kSlots * (kABlock / 2); t += kABlock) accl[t] = 0.0;
  __syncthreads();
  adjoint_sums<NPI, ROT, TAB, true>(ec, ae, sc, as, n_site, 0, ec.n, kABlock, accl);
  __syncthreads();
  adjoint_columns<true>(accl, n_site * kSlots, kABlock, site_acc);
  __syncthreads();
  if (tid < n_site * 4) {
    const int s = tid >> 2, m = tid & 3;
    double W = 0.0;
    for (int u = 0; u < n_site; ++u) W += site_acc[u * kSlots + kAdjW];
    // d SNR^2 along ln S0 of a site is minus that site's SNR^2
    const double dS = m < 3 ? site_acc[s * kSlots + kAdjS + m] : -site_acc[s * kSlots + kAdjW];
    // w_fisher sum Gbar dGamma + w_snr d ln SNR, d ln SNR = dSNR^2 / (2 SNR^2)
    ge[tid] = fma(a.w_fisher, site_acc[s * kSlots + kAdjT + m], a.w_snr * dS / (2.0 * W));
  }
}

__global__ __launch_bounds__(kABlock) void reduce_kernel(const double* __restrict__ terms, int64_t n,
                                                         int width, double* __restrict__ out) {
  __shared__ double red[kABlock / 64];
  const int c = blockIdx.x, tid = threadIdx.x;
  double t = 0.0;
  for (int64_t e = tid; e < n; e += kABlock) t += terms[e * width + c];
  t = wave_sum_a(t);
  if ((tid & 63) == 0) red[tid >> 6] = t;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kABlock / 64; ++w) s += red[w];
    out[c] = s;
  }
}

// ---------------------------------------------------- batched (work items)
// After the plan's set-up kernel has written EventC and SiteC: lanes
// [0, n) take one event each, the contractions of its Gbar (AdjEventC, ok = 0
// where the event is left out); lanes [n, n + n n_site) one (event, site)
// pair each, its AdjSiteC (not written for an event whose set-up failed).
template <int NPI>
__global__ __launch_bounds__(64) void adj_setup_kernel(AdjSetupArgs a) {
  constexpr int P = PhaseOnly<NPI>::P;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n_site = a.net.n_site;
  if (t < a.n) {
    const int64_t e = t;
    const EventC& ec = a.evc[e];
    const GbarOf gb{a.gbar, a.n, e, P, event_rows(a.par_mask, e)};
    int32_t ok = ec.status == 0 && (a.status == nullptr || a.status[e] == 0);
    for (int i = 0; i < P; ++i)               // gb is symmetric: the upper triangle decides
      for (int j = i; j < P; ++j)
        if (!finite(gb(i, j))) ok = 0;
    AdjEventC& ae = a.aec[e];
    adj_event_setup<NPI>(ec, gb, ae);
    ae.ok = ok;
    return;
  }
  const int64_t u = t - a.n;
  if (u >= a.n * n_site) return;
  const int64_t e = u / n_site;
  const int s = (int)(u - e * n_site);
  if (a.evc[e].status != 0 || (a.status != nullptr && a.status[e] != 0)) return;
  double p[kNparIn] = {};
  p[3] = a.par[3 * a.ld + e];
  p[6] = a.par[6 * a.ld + e];
  adj_site_setup(p, a.net.site[s], a.sic[u], a.asc[u], site_arms_on(a.active, a.ld, e, a.net, s));
}

// Two wavefronts per SIMD (the sums live in LDS, 40 KB per workgroup on
// five sites).  Larger workgroups put fewer events' constants in a compute
// unit's scalar cache but were measured slower on the mixed BBH/BNS workload.
template <int NPI, bool ROT, bool TAB>
__global__ __launch_bounds__(kABlock, 2) void adjoint_items_kernel(AdjItemsArgs a) {
  extern __shared__ double accl[];        // [n_site][kSlots][kABlock]
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  const int width = n_site * kSlots;
  // workgroup b takes item b: the plan orders its items longest first, and
  // workgroups are dispatched in order, so the shortest items come last
  const Item w = a.items[a.base + blockIdx.x];
  const int32_t e = __builtin_amdgcn_readfirstlane(w.e);
  const int32_t k0 = __builtin_amdgcn_readfirstlane(w.k0);
  const int32_t k1 = __builtin_amdgcn_readfirstlane(w.k1);
  // constants read through the constant address space: uniform, never
  // written during the kernel, so the compiler may use scalar loads
  typedef const __attribute__((address_space(4))) EventC CEventC;
  typedef const __attribute__((address_space(4))) AdjEventC CAdjEventC;
  typedef const __attribute__((address_space(4))) SiteC CSiteC;
  typedef const __attribute__((address_space(4))) AdjSiteC CAdjSiteC;
  const EventC& ec = *(const EventC*)((CEventC*)(a.evc) + e);
  const AdjEventC& ae = *(const AdjEventC*)((CAdjEventC*)(a.aec) + e);
  const SiteC* sc = (const SiteC*)((CSiteC*)(a.sic) + (int64_t)e * n_site);
  const AdjSiteC* as = (const AdjSiteC*)((CAdjSiteC*)(a.asc) + (int64_t)e * n_site);
  double* out = a.partial + (int64_t)__builtin_amdgcn_readfirstlane(w.slot) * width;
  if (!ae.ok) {                                  // left out: NaN marks the item for the combine
    if (tid < width) out[tid] = __builtin_nan("");
    return;
  }
  for (int t = tid; t < width * kABlock; t += kABlock) accl[t] = 0.0;
  __syncthreads();
  // two points per lane where both fit in the registers (the eccentric
  // instantiations spill with two and keep one)
  if (PhaseOnly<NPI>::ecc) adjoint_sums<NPI, ROT, TAB, false>(ec, ae, sc, as, n_site, k0, k1, kABlock, accl);
  else adjoint_sums2<NPI, ROT, TAB>(ec, ae, sc, as, n_site, k0, k1, kABlock, accl);
  __syncthreads();
  adjoint_columns<false>(accl, width, kABlock, out);
}

// One lane per event: its items' sums in item order, then the gradient terms.
__global__ void adjoint_combine_kernel(AdjCombineArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n) return;
  const int width = a.n_site * kSlots;
  const int32_t i0 = a.item_first[e], i1 = a.item_first[e + 1];
  double W = 0.0;
  for (int s = 0; s < a.n_site; ++s)
    for (int32_t i = i0; i < i1; ++i) W += a.partial[(int64_t)i * width + s * kSlots + 7];
  const bool ok = W > 0.0 && finite(W);
  double* ge = a.grad_event + e * (int64_t)(a.n_site * 4);
  for (int s = 0; s < a.n_site; ++s) {
    double t[kSlots];
#pragma unroll
    for (int m = 0; m < kSlots; ++m) t[m] = 0.0;
    for (int32_t i = i0; i < i1; ++i)
#pragma unroll
      for (int m = 0; m < kSlots; ++m) t[m] += a.partial[(int64_t)i * width + s * kSlots + m];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      // d SNR^2 along ln S0 of a site is minus that site's SNR^2
      const double dS = m < 3 ? t[4 + m] : -t[7];
      ge[s * 4 + m] = ok ? fma(a.w_fisher, t[m], a.w_snr * dS / (2.0 * W)) : 0.0;
    }
  }
}

}  // namespace

template <int NPI, bool ROT>
void launch_adjoint_items_r(const AdjItemsArgs& a, bool tab, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  if (tab) hipLaunchKernelGGL((adjoint_items_kernel<NPI, ROT, true>), grid, block, lds, s, a);
  else hipLaunchKernelGGL((adjoint_items_kernel<NPI, ROT, false>), grid, block, lds, s, a);
}

template <int NPI>
void launch_adjoint_items_n(const AdjItemsArgs& a, bool rot, bool tab, dim3 grid, dim3 block, size_t lds,
                            hipStream_t s) {
  if (rot) launch_adjoint_items_r<NPI, true>(a, tab, grid, block, lds, s);
  else launch_adjoint_items_r<NPI, false>(a, tab, grid, block, lds, s);
}

hipError_t launch_adjoint_setup(const AdjSetupArgs& a, int npi, hipStream_t s) {
  const int64_t lanes = a.n * (1 + (int64_t)a.net.n_site);
  const dim3 grid((unsigned)((lanes + 63) / 64)), block(64);
  switch (npi) {
    case 6: hipLaunchKernelGGL((adj_setup_kernel<6>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((adj_setup_kernel<5>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((adj_setup_kernel<4>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((adj_setup_kernel<3>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_items(const AdjItemsArgs& a0, int npi, bool rot, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)a0.net.n_site * kSlots * kABlock;
  const bool tab = net_has_tables(a0.net);
  return launch_slices(a0, a0.n_items, 1, kABlock, [&](const AdjItemsArgs& a, dim3 grid, dim3 block) {
    switch (npi) {
      case 6: launch_adjoint_items_n<6>(a, rot, tab, grid, block, lds, s); break;
      case 5: launch_adjoint_items_n<5>(a, rot, tab, grid, block, lds, s); break;
      case 4: launch_adjoint_items_n<4>(a, rot, tab, grid, block, lds, s); break;
      default: launch_adjoint_items_n<3>(a, rot, tab, grid, block, lds, s);
    }
  });
}

hipError_t launch_adjoint_combine(const AdjCombineArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(adjoint_combine_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int width = a.n_site * 4;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)width), dim3(kABlock), 0, s, a.grad_event, a.n, width, a.grad);
  return hipGetLastError();
}

size_t adjoint_event_bytes() { return sizeof(AdjEventC); }
size_t adjoint_site_bytes() { return sizeof(AdjSiteC); }

template <int NPI, bool ROT>
void launch_adjoint_r(const AdjointArgs& a, bool tab, dim3 grid, dim3 block, size_t lds, hipStream_t stream) {
  if (tab) hipLaunchKernelGGL((adjoint_kernel<NPI, ROT, true>), grid, block, lds, stream, a);
  else hipLaunchKernelGGL((adjoint_kernel<NPI, ROT, false>), grid, block, lds, stream, a);
}

template <int NPI>
void launch_adjoint_n(const AdjointArgs& a, bool rot, bool tab, dim3 grid, dim3 block, size_t lds,
                      hipStream_t stream) {
  if (rot) launch_adjoint_r<NPI, true>(a, tab, grid, block, lds, stream);
  else launch_adjoint_r<NPI, false>(a, tab, grid, block, lds, stream);
}

hipError_t launch_adjoint(const AdjointArgs& a0, int npi, bool rot, hipStream_t stream) {
  const size_t lds = sizeof(double) * (size_t)a0.net.n_site * kSlots * (kABlock / 2);
  const bool tab = net_has_tables(a0.net);
  hipError_t err = launch_slices(a0, a0.n, 1, kABlock, [&](const AdjointArgs& a, dim3 grid, dim3 block) {
    switch (npi) {
      case 6: launch_adjoint_n<6>(a, rot, tab, grid, block, lds, stream); break;
      case 5: launch_adjoint_n<5>(a, rot, tab, grid, block, lds, stream); break;
      case 4: launch_adjoint_n<4>(a, rot, tab, grid, block, lds, stream); break;
      default: launch_adjoint_n<3>(a, rot, tab, grid, block, lds, stream);
    }
  });
  if (err != hipSuccess) return err;
  const int width = a0.net.n_site * 4;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)width), dim3(kABlock), 0, stream, a0.grad_event, a0.n, width,
                     a0.grad);
  return hipGetLastError();
}

}  // namespace gwf

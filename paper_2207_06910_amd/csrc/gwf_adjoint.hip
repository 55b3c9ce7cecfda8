// gwf_adjoint.hip -- the adjoint (backward) pass of the Fisher/SNR map with
// respect to the detector parameters; the per-point mathematics and its
// derivation are in gwf_adjoint.hpp.
//
//   adjoint_kernel  one workgroup per event: the event's constants, its
//                   symmetrised Gbar and the sites' constants with their
//                   tangents in LDS; every lane walks the grid with a stride
//                   of the workgroup size, forms the point quantities once
//                   and, for each site, recomputes the derivative vectors and
//                   contracts them into that site's sums; each pair of lanes
//                   adds its two contributions and keeps the running sums in
//                   one LDS column (sized by the number of sites, so that two
//                   wavefronts fit per SIMD); the sums are reduced over the
//                   workgroup in a fixed order and combined into the event's
//                   gradient terms.
//   reduce_kernel   one workgroup per output component sums the events'
//                   terms in a fixed order, so the gradient is bitwise
//                   reproducible.
//
// The batched form (gwf_plan_adjoint) runs the same per-point mathematics
// over a plan's work items:
//   adjoint_items_kernel    one workgroup of 256 lanes per work item (event,
//                   point range), in the plan's longest-first order; the
//                   event's constants (from the plan's workspace), the
//                   symmetrised Gbar and the sites' constants go to LDS, each
//                   group of four lanes keeps its running per-site sums in one
//                   LDS column, and the item's sums are written to its slot
//                   (deterministic: fixed reduction order, slots in event
//                   order);
//   adjoint_combine_kernel  one lane per event sums its items' slots in item
//                   order and forms the event's gradient terms; the
//                   reduce_kernel then sums the events.
#include "gwf_adjoint.hpp"
#include "gwf_batched.hpp"
#include "gwf_kernels.hpp"

namespace gwf {

namespace {

constexpr int kABlock = 128;
constexpr int kCols = kABlock / 2;        // LDS accumulator columns, one per lane pair
// accumulator slots kept per (site, lane pair) in LDS: the four Gbar:dGamma
// terms, the three geometric SNR^2 derivatives and the site's SNR^2 (its
// ln S0 derivative is minus that)
constexpr int kSlots = 8;

__device__ inline double wave_sum_a(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ inline int slot_of(int i) { return i < 7 ? i : kAdjW; }   // LDS slot -> acc index

// Two wavefronts per SIMD: the registers are capped at 256 (the sums live in
// LDS, not in registers).
template <int NPI, bool ROT>
__global__ __launch_bounds__(kABlock, 2) void adjoint_kernel(AdjointArgs a) {
  using PO = PhaseOnly<NPI>;
  constexpr int P = PO::P;
  constexpr bool TIDAL = PO::tidal;
  constexpr uint32_t flags = (TIDAL ? kFlagTidal : 0u) | (ROT ? kFlagRot : 0u) | (PO::ecc ? kFlagEcc : 0u);
  __shared__ EventC ec;
  __shared__ SiteA sa[kMaxSites];
  __shared__ double Gb[P * P];
  extern __shared__ double accl[];      // [n_site][kSlots][kCols], column tid/2 per lane pair
  __shared__ double site_acc[kMaxSites][kSlots];
  __shared__ int32_t ok;
  const int64_t e = a.base + blockIdx.x;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  if (tid == 0) {
    double p[kNparIn];
    for (int r = 0; r < 13; ++r) p[r] = (r < 11 || TIDAL) ? a.par[r * a.ld + e] : 0.0;
    p[13] = PO::ecc && a.ecc ? a.ecc[e] : 0.0;
    p[14] = PO::ecc && a.fref ? a.fref[e] : 0.0;
    event_setup(p, a.fmin[e], a.fmax ? a.fmax[e] : 0.0, a.npts[e], flags, ec);
    ok = ec.status == 0 && (a.status == nullptr || a.status[e] == 0);
  }
  __syncthreads();
  const uint32_t pm = event_rows(a.par_mask, e);
  for (int t = tid; t < P * P; t += kABlock) {
    const int i = t / P, j = t - i * P;
    const double g = rows_in(pm, i, j)
        ? 0.5 * (a.gbar[(int64_t)(i * P + j) * a.n + e] + a.gbar[(int64_t)(j * P + i) * a.n + e]) : 0.0;
    Gb[t] = g;
    if (!finite(g)) ok = 0;          // every writer stores the same value
  }
  __syncthreads();
  double* ge = a.grad_event + e * (int64_t)(n_site * 4);
  if (!ok) {
    if (tid < n_site * 4) ge[tid] = 0.0;
    return;
  }
  if (tid < n_site) {
    double p[kNparIn];
    for (int r = 0; r < 13; ++r) p[r] = (r < 11 || TIDAL) ? a.par[r * a.ld + e] : 0.0;
    site_setup_adj(p, a.net.site[tid], ec, sa[tid], site_arms_on(a.active, a.ld, e, a.net, tid));
  }
  const int col = tid >> 1;
  if ((tid & 1) == 0)
    for (int s = 0; s < n_site; ++s)
#pragma unroll
      for (int i = 0; i < kSlots; ++i) accl[(s * kSlots + i) * kCols + col] = 0.0;
  __syncthreads();
  // every lane walks its grid points once (the same trip count for every
  // lane, so that both lanes of a pair take part in each exchange; points
  // past the grid add zero); the point quantities are shared by all sites
  const int iters = (ec.n + kABlock - 1) / kABlock;
  for (int it = 0; it < iters; ++it) {
    asm volatile("" ::: "memory");   // constants stay in LDS rather than occupying registers
    const int k = it * kABlock + tid;
    const bool in = k < ec.n;
    AdjPoint ap;
    if (in) adjoint_point_setup<NPI, ROT>(ec, Gb, k, ap);
    for (int s = 0; s < n_site; ++s) {
      asm volatile("" ::: "memory");
      double acc[kAdjN];
#pragma unroll
      for (int i = 0; i < kAdjN; ++i) acc[i] = 0.0;
      if (in) adjoint_site<NPI>(ec, sa[s], Gb, ap, acc);
#pragma unroll
      for (int i = 0; i < kSlots; ++i) {
        const double v = acc[slot_of(i)];
        const double t = v + __shfl_xor(v, 1, 64);       // the lane pair's two points
        if ((tid & 1) == 0) accl[(s * kSlots + i) * kCols + col] += t;
      }
    }
  }
  __syncthreads();
  // the first wavefront sums the columns (kCols = 64 lanes)
  if (tid < kCols) {
    for (int s = 0; s < n_site; ++s)
#pragma unroll
      for (int i = 0; i < kSlots; ++i) {
        const double t = wave_sum_a(accl[(s * kSlots + i) * kCols + tid]);
        if (tid == 0) site_acc[s][i] = t;
      }
  }
  __syncthreads();
  if (tid < n_site * 4) {
    const int s = tid >> 2, m = tid & 3;
    double W = 0.0;
    for (int u = 0; u < n_site; ++u) W += site_acc[u][7];
    // d SNR^2 along ln S0 of a site is minus that site's SNR^2
    const double dS = m < 3 ? site_acc[s][4 + m] : -site_acc[s][7];
    // w_fisher sum Gbar dGamma + w_snr d ln SNR, d ln SNR = dSNR^2 / (2 SNR^2)
    ge[tid] = fma(a.w_fisher, site_acc[s][m], a.w_snr * dS / (2.0 * W));
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
constexpr int kAIBlock = 256;
constexpr int kAICols = kAIBlock / 4;     // LDS accumulator columns, one per group of four lanes

template <int NPI, bool ROT>
__global__ __launch_bounds__(kAIBlock, 2) void adjoint_items_kernel(AdjItemsArgs a) {
  constexpr int P = PhaseOnly<NPI>::P;
  __shared__ double Gb[P * P];
  __shared__ SiteA sa[kMaxSites];
  __shared__ EventC ec;
  extern __shared__ double accl[];        // [n_site][kSlots][kAICols]
  __shared__ int32_t ok;
  const int tid = threadIdx.x;
  const int n_site = a.net.n_site;
  const int col = tid >> 2;
  const int width = n_site * kSlots;
  // workgroup b takes item b: the plan orders its items longest first, and
  // workgroups are dispatched in order, so the shortest items come last
  const Item w = a.items[a.base + blockIdx.x];
  const int32_t e = __builtin_amdgcn_readfirstlane(w.e);
  const int32_t k0 = __builtin_amdgcn_readfirstlane(w.k0);
  const int32_t k1 = __builtin_amdgcn_readfirstlane(w.k1);
  // the event's constants from the plan's workspace into LDS (re-read there
  // at every use rather than held in registers)
  {
    static_assert(sizeof(EventC) % sizeof(double) == 0, "EventC copied as doubles");
    const double* src = reinterpret_cast<const double*>(a.evc + e);
    double* dst = reinterpret_cast<double*>(&ec);
    for (int t = tid; t < (int)(sizeof(EventC) / sizeof(double)); t += kAIBlock) dst[t] = src[t];
  }
  double* out = a.partial + (int64_t)__builtin_amdgcn_readfirstlane(w.slot) * width;
  __syncthreads();
  if (tid == 0) ok = ec.status == 0 && (a.status == nullptr || a.status[e] == 0);
  __syncthreads();
  const uint32_t pm = event_rows(a.par_mask, e);
  for (int t = tid; t < P * P; t += kAIBlock) {
    const int i = t / P, j = t - i * P;
    const double g = rows_in(pm, i, j)
        ? 0.5 * (a.gbar[(int64_t)(i * P + j) * a.n + e] + a.gbar[(int64_t)(j * P + i) * a.n + e]) : 0.0;
    Gb[t] = g;
    if (!finite(g)) ok = 0;                     // every writer stores the same value
  }
  if (tid < n_site) {
    double p[kNparIn] = {};
    p[3] = a.par[3 * a.ld + e];
    p[4] = a.par[4 * a.ld + e];
    p[6] = a.par[6 * a.ld + e];
    site_setup_adj(p, a.net.site[tid], ec, sa[tid], site_arms_on(a.active, a.ld, e, a.net, tid));
  }
  for (int t = tid; t < width * kAICols; t += kAIBlock) accl[t] = 0.0;
  __syncthreads();
  if (!ok) {                                     // left out: NaN marks the item for the combine
    if (tid < width) out[tid] = __builtin_nan("");
    return;
  }
  const int iters = (k1 - k0 + kAIBlock - 1) / kAIBlock;   // same trip count for every lane
  for (int r = 0; r < iters; ++r) {
    asm volatile("" ::: "memory");
    const int k = k0 + r * kAIBlock + tid;
    const bool in = k < k1;
    AdjPoint ap;
    if (in) adjoint_point_setup<NPI, ROT>(ec, Gb, k, ap);
    for (int s = 0; s < n_site; ++s) {
      asm volatile("" ::: "memory");
      double acc[kAdjN];
#pragma unroll
      for (int i = 0; i < kAdjN; ++i) acc[i] = 0.0;
      if (in) adjoint_site<NPI>(ec, sa[s], Gb, ap, acc);
#pragma unroll
      for (int i = 0; i < kSlots; ++i) {
        double v = acc[slot_of(i)];
        v += __shfl_xor(v, 1, 64);               // the group's four points
        v += __shfl_xor(v, 2, 64);
        if ((tid & 3) == 0) accl[(s * kSlots + i) * kAICols + col] += v;
      }
    }
  }
  __syncthreads();
  if (tid < kAICols) {                           // the first wavefront sums the 64 columns
    for (int t = 0; t < width; ++t) {
      const double v = wave_sum_a(accl[t * kAICols + tid]);
      if (tid == 0) out[t] = v;
    }
  }
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

template <int NPI>
void launch_adjoint_items_n(const AdjItemsArgs& a, bool rot, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  if (rot) hipLaunchKernelGGL((adjoint_items_kernel<NPI, true>), grid, block, lds, s, a);
  else hipLaunchKernelGGL((adjoint_items_kernel<NPI, false>), grid, block, lds, s, a);
}

hipError_t launch_adjoint_items(const AdjItemsArgs& a0, int npi, bool rot, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)a0.net.n_site * kSlots * kAICols;
  return launch_slices(a0, a0.n_items, 1, kAIBlock, [&](const AdjItemsArgs& a, dim3 grid, dim3 block) {
    switch (npi) {
      case 6: launch_adjoint_items_n<6>(a, rot, grid, block, lds, s); break;
      case 5: launch_adjoint_items_n<5>(a, rot, grid, block, lds, s); break;
      case 4: launch_adjoint_items_n<4>(a, rot, grid, block, lds, s); break;
      default: launch_adjoint_items_n<3>(a, rot, grid, block, lds, s);
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

int adjoint_items_block() { return kAIBlock; }

template <int NPI>
void launch_adjoint_n(const AdjointArgs& a, bool rot, dim3 grid, dim3 block, size_t lds, hipStream_t stream) {
  if (rot) hipLaunchKernelGGL((adjoint_kernel<NPI, true>), grid, block, lds, stream, a);
  else hipLaunchKernelGGL((adjoint_kernel<NPI, false>), grid, block, lds, stream, a);
}

hipError_t launch_adjoint(const AdjointArgs& a0, int npi, bool rot, hipStream_t stream) {
  const size_t lds = sizeof(double) * (size_t)a0.net.n_site * kSlots * kCols;
  hipError_t err = launch_slices(a0, a0.n, 1, kABlock, [&](const AdjointArgs& a, dim3 grid, dim3 block) {
    switch (npi) {
      case 6: launch_adjoint_n<6>(a, rot, grid, block, lds, stream); break;
      case 5: launch_adjoint_n<5>(a, rot, grid, block, lds, stream); break;
      case 4: launch_adjoint_n<4>(a, rot, grid, block, lds, stream); break;
      default: launch_adjoint_n<3>(a, rot, grid, block, lds, stream);
    }
  });
  if (err != hipSuccess) return err;
  const int width = a0.net.n_site * 4;
  hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)width), dim3(kABlock), 0, stream, a0.grad_event, a0.n, width,
                     a0.grad);
  return hipGetLastError();
}

}  // namespace gwf

// gwf_batched.hip -- batched form of the Fisher/SNR path for catalogues with
// uneven grid lengths.
//
//   setup_kernel    one lane per event and one per event x site: the
//                   per-event and per-site constants, written once to a
//                   workspace.
//   items_kernel    one workgroup per work item (event, point range [k0, k1),
//                   at most `chunk` points), dispatched in the plan's
//                   longest-first order, writes the item's partial sums to its
//                   own slot (the item's position in event order), so long
//                   and short events are spread evenly over the chip, the
//                   last items to start are the shortest, and the result
//                   does not depend on which workgroup took which item.  (A
//                   persistent form pulling items from a counter kept more
//                   values live across its outer loop: more register spills,
//                   1.7% slower.)  The event's constants are read from the
//                   workspace through the constant address space, i.e. by
//                   scalar loads into SGPRs, which costs neither LDS traffic
//                   nor vector registers.
//   combine_kernel  sums each event's item partials in item order and writes
//                   the Fisher matrix, SNR and status.
// Every step is an ordinary kernel on one stream, so the sequence can be
// captured in a HIP graph and replayed.
#include "gwf_batched.hpp"
#include "gwf_fisher_body.hpp"

namespace gwf {

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Lanes [0, n) take one event each (EventC and its status), lanes
// [n, n + n n_site) one (event, site) pair each (SiteC, with pi M formed from
// the parameters exactly as the event's lane forms it); both write straight
// into the workspace.  A site of an event whose set-up fails is written
// anyway and never read.
__global__ __launch_bounds__(64) void setup_kernel(SetupArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n_site = a.net.n_site;
  if (t >= a.n * (1 + n_site)) return;
  const int64_t e = t < a.n ? t : (t - a.n) / n_site;
  const bool tidal = (a.flags & kFlagTidal) != 0;
  double p[kNparIn];
  for (int r = 0; r < 13; ++r) p[r] = (r < 11 || tidal) ? a.par[r * a.ld + e] : 0.0;
  p[13] = (a.flags & kFlagEcc) && a.ecc ? a.ecc[e] : 0.0;
  p[14] = (a.flags & kFlagEcc) && a.fref ? a.fref[e] : 0.0;
  if (t < a.n) {
    EventC& ec = a.evc[e];
    event_setup(p, a.fmin[e], a.fmax ? a.fmax[e] : 0.0, a.npts[e], a.flags, ec);
    if (!ec.status && (a.npts[e] != a.npts_plan[e] || a.npts[e] > a.npts_max))
      ec.status = kEvInvalid;   // grid changed since the items were built, or longer than they allow
    if (a.status) a.status[e] = ec.status;
    return;
  }
  const int s = (int)(t - a.n - e * n_site);
  site_setup(p, a.net.site[s], kPi * total_mass_s(p), a.sic[e * n_site + s],
             site_arms_on(a.active, a.ld, e, a.net, s));
}

template <int NPI, bool ROT, bool MIXED, bool TAB>
__global__ __launch_bounds__(FisherDims<NPI>::TIDAL ? 2 * kBlock : kBlock) void items_kernel(ItemsArgs a) {
  using Dm = FisherDims<NPI>;
  constexpr int NACC = Dm::NACC;
  __shared__ FisherLds L;
  const int tid = threadIdx.x;
  const int n_site = a.n_site;
  // workgroup b takes item b (the plan orders its items longest first, and
  // workgroups are dispatched in order); with the count on the device, the
  // grid is its upper bound and the surplus workgroups leave
  const int32_t n_items = a.n_items_dev ? *a.n_items_dev : a.n_items;
  const int64_t it = a.base + blockIdx.x;
  if (it >= n_items) return;
  const Item w = a.items[it];
  const int32_t ew = __builtin_amdgcn_readfirstlane(w.e);
  const int32_t k0 = __builtin_amdgcn_readfirstlane(w.k0);
  const int32_t k1 = __builtin_amdgcn_readfirstlane(w.k1);
  // constants read through the constant address space: uniform, never
  // written during the kernel, so the compiler may use scalar loads
  typedef const __attribute__((address_space(4))) EventC CEventC;
  typedef const __attribute__((address_space(4))) SiteC CSiteC;
  CEventC* ecp = (CEventC*)(a.evc) + ew;
  CSiteC* scp = (CSiteC*)(a.sic) + (int64_t)ew * n_site;
  const EventC& ecg = *(const EventC*)ecp;
  const SiteC* scg = (const SiteC*)scp;
  double* out = a.partial + (int64_t)__builtin_amdgcn_readfirstlane(w.slot) * NACC;
  if (ecg.status) {
    if (tid < NACC) out[tid] = 0.0;
  } else {
    double t = 0.0;
    // both forms: PN series as sums of products over shared powers and the
    // PSD power law once per point (in FP32 for the mixed form)
    fisher_sums<NPI, ROT, MIXED, true, false, TAB>(ecg, scg, n_site, k0, k1, L, &t);
    if (tid < NACC) out[tid] = t;
  }
}

template <int NPI_>
__global__ void combine_kernel(CombineArgs a) {
  using Dm = FisherDims<NPI_>;
  constexpr int P = Dm::P, NPI = Dm::NPI, NACC = Dm::NACC;
  const int64_t t = a.base + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n * NACC) return;
  const int64_t e = t / NACC;
  const int slot = (int)(t - e * NACC);
  const int32_t st0 = a.evc[e].status;
  double s = 0.0;
  if (!st0)
    for (int32_t i = a.item_first[e]; i < a.item_first[e + 1]; ++i) s += a.partial[(int64_t)i * NACC + slot];
  int r, c;
  slot_position(slot, NPI, r, c);
  if (r == 8 && c == 8) a.snr[e] = sqrt(s);
  if (!rows_in(event_rows(a.par_mask, e), r, c)) s = 0.0;   // not one of the event's rows
  a.fisher[((int64_t)r * P + c) * a.n + e] = s;
  a.fisher[((int64_t)c * P + r) * a.n + e] = s;
  // the set-up kernel wrote the parameter status; a non-finite sum adds its bit
  if (!st0 && !finite(s)) atomicOr(a.status + e, (int32_t)kEvNonFinite);
}

constexpr int kScanBlock = 1024;

// One workgroup: item counts per event and their exclusive prefix sum, tile
// by tile of kScanBlock events (wavefront scans, then the wavefront totals,
// then the running carry of the earlier tiles).
__global__ __launch_bounds__(kScanBlock) void items_scan_kernel(const int32_t* __restrict__ npts, int64_t n,
                                                                int32_t chunk, int32_t npts_max,
                                                                int32_t* __restrict__ first,
                                                                int32_t* __restrict__ n_items) {
  __shared__ int32_t wtot[kScanBlock / 64];
  __shared__ int32_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += kScanBlock) {
    const int64_t e = base + tid;
    int32_t c = 0;
    if (e < n) {
      int32_t m = npts[e];
      if (m < 2 || m > npts_max) m = 2;
      c = (m - 1) / chunk + 1;
    }
    int32_t x = c;                                   // inclusive scan within the wavefront
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    int32_t before = carry;                          // earlier tiles and earlier wavefronts
    for (int w = 0; w < wave; ++w) before += wtot[w];
    if (e < n) first[e] = before + x - c;
    __syncthreads();                                 // every lane has read carry and wtot
    if (tid == kScanBlock - 1) carry = before + x;
    __syncthreads();
  }
  if (tid == 0) {
    first[n] = carry;
    *n_items = carry;
  }
}

// One lane per event writes its items (slot = position in event order).
__global__ void items_fill_kernel(const int32_t* __restrict__ npts, int64_t n, int32_t chunk, int32_t npts_max,
                                  const int32_t* __restrict__ first, Item* __restrict__ items) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  int32_t m = npts[e];
  if (m < 2 || m > npts_max) m = 2;
  const int32_t f0 = first[e], f1 = first[e + 1];
  for (int32_t i = f0, k0 = 0; i < f1; ++i, k0 += chunk)
    items[i] = Item{(int32_t)e, k0, min(m, k0 + chunk), i};
}

hipError_t launch_items_build(const int32_t* npts, int64_t n, int32_t chunk, int32_t npts_max, int32_t* first,
                              int32_t* n_items, Item* items, hipStream_t s) {
  hipLaunchKernelGGL(items_scan_kernel, dim3(1), dim3(kScanBlock), 0, s, npts, n, chunk, npts_max, first, n_items);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(items_fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, npts, n, chunk, npts_max,
                     first, items);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_setup(const SetupArgs& a, hipStream_t s) {
  const int64_t lanes = a.n * (1 + (int64_t)a.net.n_site);
  hipLaunchKernelGGL(setup_kernel, dim3((unsigned)((lanes + 63) / 64)), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <int NPI, bool MIXED>
void launch_items_n(const ItemsArgs& a, bool rot, bool tab, dim3 grid, dim3 block, hipStream_t s) {
  if (rot && tab) hipLaunchKernelGGL((items_kernel<NPI, true, MIXED, true>), grid, block, 0, s, a);
  else if (rot) hipLaunchKernelGGL((items_kernel<NPI, true, MIXED, false>), grid, block, 0, s, a);
  else if (tab) hipLaunchKernelGGL((items_kernel<NPI, false, MIXED, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((items_kernel<NPI, false, MIXED, false>), grid, block, 0, s, a);
}

template <bool MIXED>
void launch_items_t(const ItemsArgs& a, int npi, bool rot, bool tab, dim3 grid, dim3 block, hipStream_t s) {
  switch (npi) {
    case 6: launch_items_n<6, MIXED>(a, rot, tab, grid, block, s); break;
    case 5: launch_items_n<5, MIXED>(a, rot, tab, grid, block, s); break;
    case 4: launch_items_n<4, MIXED>(a, rot, tab, grid, block, s); break;
    default: launch_items_n<3, MIXED>(a, rot, tab, grid, block, s);
  }
}

hipError_t launch_items(const ItemsArgs& a0, int npi, bool rot, bool mixed, bool tab, int64_t n_wg, hipStream_t s) {
  return launch_slices(a0, n_wg, 1, kBlock, [&](const ItemsArgs& a, dim3 grid, dim3 block) {
    if (mixed) launch_items_t<true>(a, npi, rot, tab, grid, block, s);
    else launch_items_t<false>(a, npi, rot, tab, grid, block, s);
  });
}

int fisher_nacc(int npi) {
  switch (npi) {
    case 6: return FisherDims<6>::NACC;
    case 5: return FisherDims<5>::NACC;
    case 4: return FisherDims<4>::NACC;
    default: return FisherDims<3>::NACC;
  }
}

hipError_t launch_combine(const CombineArgs& a0, int npi, hipStream_t s) {
  return launch_slices(a0, a0.n * fisher_nacc(npi), 256, 256, [&](const CombineArgs& a, dim3 grid, dim3 block) {
    switch (npi) {
      case 6: hipLaunchKernelGGL((combine_kernel<6>), grid, block, 0, s, a); break;
      case 5: hipLaunchKernelGGL((combine_kernel<5>), grid, block, 0, s, a); break;
      case 4: hipLaunchKernelGGL((combine_kernel<4>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((combine_kernel<3>), grid, block, 0, s, a);
    }
  });
}

int fisher_block() { return kBlock; }

}  // namespace gwf

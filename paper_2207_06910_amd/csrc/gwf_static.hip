// gwf_static.hip -- gwf_fisher_static: the batched form of the Fisher/SNR
// path (work items of at most `chunk` points, one workgroup each, partial
// sums combined per event in item order) for callers that cannot allocate
// device memory.  Its workspace -- the per-event and per-site constants, the
// work items, their count and their partial sums -- lives in one file-scope
// device array of fixed size instead of a
// plan's allocations, and the work items are built on the device from the
// grid lengths, so the call neither allocates nor reads anything back.
//
// The kernels are those of the plan (gwf_batched.hip) with the items built
// by launch_items_build; the items are taken in slot order rather than
// longest first, by a grid of the largest item count the workspace allows
// (workgroups beyond the count built on the device leave at once).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "../../include/gwf.h"
#include "gwf_api_internal.hpp"
#include "gwf_batched.hpp"

using namespace gwf;

static_assert(GWF_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size");

// The workspace of every gwf_fisher_static call on a device: one copy per
// device, held from the library's load until the process ends.
static __device__ __align__(256) unsigned char scratch[GWF_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = GWF_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Its device address on each device, looked up once per device (the name
// `scratch` in host code is only a host-side stand-in for the symbol).
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gwf_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return api_fail(GWF_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !p) return api_hip_fail(err != hipSuccess ? err : hipErrorInvalidSymbol, "scratch symbol address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GWF_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" {

gwf_status gwf_fisher_static(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                             uint32_t flags, int32_t chunk, int32_t npts_max, double* fisher, double* snr,
                             int32_t* status, void* stream) {
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (grid->kind == GWF_GRID_EXPLICIT)
    return api_fail(GWF_E_UNSUPPORTED, "the batched form generates log grids; use gwf_fisher for explicit grids");
  if (!fisher || !snr || !status) return api_fail(GWF_E_INVALID_ARG, "fisher, snr and status are required");
  if (chunk < 256 || chunk > (1 << 30) || chunk % fisher_block() != 0)
    return api_fail(GWF_E_INVALID_ARG, "chunk=%d must be a positive multiple of %d", chunk, fisher_block());
  if (npts_max < 2 || npts_max > (1 << 30)) return api_fail(GWF_E_INVALID_ARG, "npts_max=%d outside 2..2^30", npts_max);
  NetDesc nd;
  if ((st = api_pack_network(net, nd))) return st;
  const bool rot = (flags & GWF_EARTH_ROT) != 0, mixed = (flags & GWF_MIXED) != 0;
  const int npi = api_npi(flags);
  const int nacc = fisher_nacc(npi);
  // workspace layout, each part 256-byte aligned
  const int64_t n = ev->n;
  const int64_t per_event = (npts_max - 1) / chunk + 1;
  const int64_t items_max = n * per_event;
  const size_t o_evc = 0;
  const size_t o_sic = o_evc + align256((size_t)n * sizeof(EventC));
  const size_t o_first = o_sic + align256((size_t)n * nd.n_site * sizeof(SiteC));
  const size_t o_items = o_first + align256((size_t)(n + 1) * sizeof(int32_t));
  const size_t o_part = o_items + align256((size_t)items_max * sizeof(Item));
  const size_t o_cnt = o_part + align256((size_t)items_max * nacc * sizeof(double));
  const size_t need = o_cnt + 256;
  if (items_max > 0x7fffffffLL || need > kScratchBytes)
    return api_fail(GWF_E_INVALID_ARG,
                    "%lld events with grids up to %d points in items of %d need %zu bytes of workspace, more "
                    "than the %zu of gwf_fisher_static (use a plan)",
                    (long long)n, npts_max, chunk, need, kScratchBytes);
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return api_hip_fail(err, "hipGetDevice");
  void* base = nullptr;
  if ((st = scratch_address(dev, &base))) return st;
  unsigned char* w = static_cast<unsigned char*>(base);
  EventC* evc = reinterpret_cast<EventC*>(w + o_evc);
  SiteC* sic = reinterpret_cast<SiteC*>(w + o_sic);
  int32_t* first = reinterpret_cast<int32_t*>(w + o_first);
  Item* items = reinterpret_cast<Item*>(w + o_items);
  double* partial = reinterpret_cast<double*>(w + o_part);
  int32_t* n_items = reinterpret_cast<int32_t*>(w + o_cnt);
  hipStream_t s = (hipStream_t)stream;
  // items from the grid lengths
  err = launch_items_build(grid->npts, n, chunk, npts_max, first, n_items, items, s);
  if (err == hipSuccess) {
    SetupArgs sa{};
    sa.par = ev->par; sa.ld = ev->ld; sa.n = n;
    sa.fmin = grid->fmin; sa.fmax = grid->fmax; sa.npts = grid->npts; sa.npts_plan = grid->npts;
    sa.npts_max = npts_max;
    sa.ecc = ev->ecc; sa.fref = ev->f_ref_ecc;
    sa.net = nd; sa.flags = flags; sa.evc = evc; sa.sic = sic; sa.status = status;
    sa.active = ev->active;
    err = launch_setup(sa, s);
  }
  if (err == hipSuccess) {
    ItemsArgs ia{};
    ia.evc = evc; ia.sic = sic; ia.n_site = nd.n_site; ia.items = items;
    ia.n_items = 0; ia.n_items_dev = n_items; ia.partial = partial;
    err = launch_items(ia, npi, rot, mixed, net_has_tables(nd), std::max<int64_t>(items_max, 1), s);
  }
  if (err == hipSuccess) {
    CombineArgs ca{};
    ca.n = n; ca.evc = evc; ca.item_first = first; ca.partial = partial;
    ca.fisher = fisher; ca.snr = snr; ca.status = status; ca.par_mask = ev->par_mask;
    err = launch_combine(ca, npi, s);
  }
  if (err != hipSuccess) return api_hip_fail(err, "gwf_fisher_static launch");
  return GWF_OK;
}

}  // extern "C"

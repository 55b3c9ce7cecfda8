// gwf_plan.hip -- host side of the batched form (gwf_plan_* in include/gwf.h):
// work-item tables, workspace, autotuning of the item length, and
// capture/replay of the whole
// set-up -> items -> combine (-> inversion) sequence as one HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gwf.h"
#include "gwf_api_internal.hpp"
#include "gwf_batched.hpp"

using namespace gwf;

struct gwf_plan {
  gwf_events ev{};
  gwf_grid grid{};
  NetDesc net{};
  uint32_t flags = 0;
  int64_t n = 0;
  int P = 0, npi = 3, nacc = 0, n_site_alloc = 0;
  bool tidal = false, rot = false, mixed = false, tab = false;
  std::vector<int32_t> npts_host;
  // tuning
  int chunk = 0, n_items = 0;
  bool use_graph = true;
  int32_t inv_method = GWF_INV_CHO;
  double tuned_ms = 0.0;
  // workspace
  EventC* evc = nullptr;
  SiteC* sic = nullptr;
  int32_t* npts_plan = nullptr;
  Item* items = nullptr;
  int32_t* item_first = nullptr;
  double* partial = nullptr;
  size_t items_cap = 0;
  // the adjoint's constants (allocated by the first gwf_plan_adjoint)
  AdjEventC* aec = nullptr;
  AdjSiteC* asc = nullptr;
  int64_t workspace_bytes = 0;
  // graph cache, keyed by the output pointers of the last replay
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[8] = {};
  double key_cond = 0.0;
  // optional timing of the work-item kernel (direct launches only)
  bool profile = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

template <class T>
hipError_t dev_alloc(T** p, size_t count, int64_t& total) {
  total += (int64_t)(count * sizeof(T));
  return hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
}

// Work items of at most `chunk` points.  Their slots (partial-sum positions)
// follow event order, so an event's items occupy slots first[e] ..
// first[e+1]-1; the processing order is longest first (ties in slot order),
// which leaves the shortest items for the end of the launch.
void build_items(const std::vector<int32_t>& npts, int chunk, std::vector<Item>& items,
                 std::vector<int32_t>& first) {
  items.clear();
  first.assign(npts.size() + 1, 0);
  for (size_t e = 0; e < npts.size(); ++e) {
    first[e] = (int32_t)items.size();
    const int32_t n = npts[e] >= 2 ? npts[e] : 2;     // invalid events still get one (skipped) item
    for (int32_t k0 = 0; k0 < n; k0 += chunk)
      items.push_back(Item{(int32_t)e, k0, std::min(n, k0 + chunk), (int32_t)items.size()});
  }
  first[npts.size()] = (int32_t)items.size();
  std::stable_sort(items.begin(), items.end(),
                   [](const Item& a, const Item& b) { return a.k1 - a.k0 > b.k1 - b.k0; });
}

gwf_status set_items(gwf_plan* p, int chunk) {
  std::vector<Item> items;
  std::vector<int32_t> first;
  build_items(p->npts_host, chunk, items, first);
  if (items.size() > 0x7fffffffull) return api_fail(GWF_E_INVALID_ARG, "too many work items");
  hipError_t err;
  if (items.size() > p->items_cap) {
    (void)hipFree(p->items);
    (void)hipFree(p->partial);
    p->items = nullptr;
    p->partial = nullptr;
    int64_t dummy = 0;
    if ((err = dev_alloc(&p->items, items.size(), dummy)) != hipSuccess ||
        (err = dev_alloc(&p->partial, items.size() * (size_t)p->nacc, dummy)) != hipSuccess)
      return api_fail(GWF_E_NOMEM, "work-item workspace (%zu items): %s", items.size(), hipGetErrorString(err));
    p->items_cap = items.size();
  }
  if ((err = hipMemcpy(p->items, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice)) != hipSuccess ||
      (err = hipMemcpy(p->item_first, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)
    return api_hip_fail(err, "work-item upload");
  p->chunk = chunk;
  p->n_items = (int)items.size();
  return GWF_OK;
}

struct Outs {
  double* fisher;
  double* snr;
  int32_t* status;
  double cond_max;
  double *cov, *sigma, *cond, *inv_err;
};

// Enqueue the whole batched path on stream s.
gwf_status enqueue(gwf_plan* p, const Outs& o, hipStream_t s) {
  SetupArgs sa{};
  sa.par = p->ev.par; sa.ld = p->ev.ld; sa.n = p->n;
  sa.fmin = p->grid.fmin; sa.fmax = p->grid.fmax; sa.npts = p->grid.npts; sa.npts_plan = p->npts_plan;
  sa.npts_max = 0x7fffffff;
  sa.ecc = p->ev.ecc; sa.fref = p->ev.f_ref_ecc;
  sa.net = p->net; sa.flags = p->flags; sa.evc = p->evc; sa.sic = p->sic; sa.status = o.status;
  sa.active = p->ev.active;
  hipError_t err = launch_setup(sa, s);
  if (err == hipSuccess) {
    ItemsArgs ia{};
    ia.evc = p->evc; ia.sic = p->sic; ia.n_site = p->net.n_site; ia.items = p->items;
    ia.n_items = p->n_items; ia.partial = p->partial;
    const bool timed = p->profile && p->ev0;
    if (timed) (void)hipEventRecord(p->ev0, s);
    err = launch_items(ia, p->npi, p->rot, p->mixed, p->tab, p->n_items, s);
    if (timed) (void)hipEventRecord(p->ev1, s);
  }
  if (err == hipSuccess) {
    CombineArgs ca{};
    ca.n = p->n; ca.evc = p->evc; ca.item_first = p->item_first; ca.partial = p->partial;
    ca.fisher = o.fisher; ca.snr = o.snr; ca.status = o.status; ca.par_mask = p->ev.par_mask;
    err = launch_combine(ca, p->npi, s);
  }
  if (err == hipSuccess && o.sigma) {
    InvertArgs ia{};
    ia.n = p->n; ia.fisher = o.fisher; ia.cond_max = o.cond_max; ia.cov = o.cov; ia.sigma = o.sigma;
    ia.cond = o.cond; ia.inv_err = o.inv_err; ia.status = o.status; ia.par_mask = p->ev.par_mask;
    ia.method = p->inv_method;
    err = launch_invert(ia, p->P, s);
  }
  if (err != hipSuccess) return api_hip_fail(err, "batched launch");
  return GWF_OK;
}

double time_config(gwf_plan* p, const Outs& o, hipStream_t s) {
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  enqueue(p, o, s);                 // warm-up
  (void)hipEventRecord(a, s);
  enqueue(p, o, s);
  (void)hipEventRecord(b, s);
  (void)hipEventSynchronize(b);
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

void free_plan(gwf_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->ev0) (void)hipEventDestroy(p->ev0);
  if (p->ev1) (void)hipEventDestroy(p->ev1);
  for (void* q : {(void*)p->evc, (void*)p->sic, (void*)p->npts_plan, (void*)p->items, (void*)p->item_first,
                  (void*)p->partial, (void*)p->aec, (void*)p->asc})
    (void)hipFree(q);
  delete p;
}

}  // namespace

extern "C" {

gwf_status gwf_plan_create(const gwf_events* ev, const gwf_network* net, const gwf_grid* grid,
                           uint32_t flags, const gwf_plan_options* opt, gwf_plan** out,
                           void* stream) {
  if (!out) return api_fail(GWF_E_INVALID_ARG, "plan output pointer is NULL");
  *out = nullptr;
  gwf_status st = api_check_common(ev, grid, flags);
  if (st) return st;
  if (grid->kind == GWF_GRID_EXPLICIT)
    return api_fail(GWF_E_UNSUPPORTED, "plans generate log grids; use gwf_fisher for explicit grids");
  gwf_plan* p = new gwf_plan();
  if ((st = api_pack_network(net, p->net))) { delete p; return st; }
  gwf_plan_options o{};
  if (opt) o = *opt; else o.use_graph = 1;
  if (o.chunk < 0 || (o.chunk % fisher_block()) != 0) {
    delete p;
    return api_fail(GWF_E_INVALID_ARG, "chunk=%d must be a non-negative multiple of %d", o.chunk, fisher_block());
  }
  if (o.inv_method != GWF_INV_CHO && o.inv_method != GWF_INV_CHO_SVD && o.inv_method != GWF_INV_CHO_DD) {
    delete p;
    return api_fail(GWF_E_INVALID_ARG, "inv_method=%d: plans invert by GWF_INV_CHO, GWF_INV_CHO_SVD or GWF_INV_CHO_DD",
                    o.inv_method);
  }
  p->ev = *ev; p->grid = *grid; p->flags = flags; p->n = ev->n;
  p->tidal = (flags & GWF_TIDAL) != 0;
  p->rot = (flags & GWF_EARTH_ROT) != 0;
  p->mixed = (flags & GWF_MIXED) != 0;
  p->tab = net_has_tables(p->net);
  p->npi = api_npi(flags);
  p->P = 8 + p->npi;
  p->nacc = fisher_nacc(p->npi);
  p->use_graph = o.use_graph != 0;
  p->inv_method = o.inv_method;
  if (o.profile && p->use_graph) {
    delete p;
    return api_fail(GWF_E_INVALID_ARG, "profile needs use_graph = 0 (kernels launched directly)");
  }
  hipStream_t s = (hipStream_t)stream;
  hipError_t err;
  // grid lengths are fixed for the life of the plan
  p->npts_host.resize(p->n);
  if ((err = hipMemcpyAsync(p->npts_host.data(), grid->npts, p->n * sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (err = hipStreamSynchronize(s)) != hipSuccess) {
    free_plan(p);
    return api_hip_fail(err, "reading grid lengths");
  }
  int64_t total = 0;
  p->n_site_alloc = p->net.n_site;
  if ((err = dev_alloc(&p->evc, p->n, total)) != hipSuccess ||
      (err = dev_alloc(&p->sic, p->n * p->net.n_site, total)) != hipSuccess ||
      (err = dev_alloc(&p->npts_plan, p->n, total)) != hipSuccess ||
      (err = dev_alloc(&p->item_first, p->n + 1, total)) != hipSuccess) {
    free_plan(p);
    return api_fail(GWF_E_NOMEM, "plan workspace: %s", hipGetErrorString(err));
  }
  if ((err = hipMemcpy(p->npts_plan, p->npts_host.data(), p->n * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess) {
    free_plan(p);
    return api_hip_fail(err, "grid-length upload");
  }
  // candidate item lengths
  std::vector<int> chunks = o.chunk ? std::vector<int>{o.chunk} : std::vector<int>{2048, 4096, 8192, 16384};
  int best_c = chunks[0];
  double best = 0.0;
  if (chunks.size() > 1) {
    double *tf = nullptr, *ts = nullptr;
    int32_t* tst = nullptr;
    int64_t dummy = 0;
    if ((err = dev_alloc(&tf, (size_t)p->P * p->P * p->n, dummy)) != hipSuccess ||
        (err = dev_alloc(&ts, p->n, dummy)) != hipSuccess || (err = dev_alloc(&tst, p->n, dummy)) != hipSuccess) {
      (void)hipFree(tf); (void)hipFree(ts); (void)hipFree(tst);
      free_plan(p);
      return api_fail(GWF_E_NOMEM, "autotune buffers: %s", hipGetErrorString(err));
    }
    Outs to{tf, ts, tst, 1e50, nullptr, nullptr, nullptr, nullptr};
    best = 1e300;
    for (int c : chunks) {
      if ((st = set_items(p, c))) { (void)hipFree(tf); (void)hipFree(ts); (void)hipFree(tst); free_plan(p); return st; }
      const double ms = time_config(p, to, s);
      if (ms < best) { best = ms; best_c = c; }
    }
    (void)hipFree(tf); (void)hipFree(ts); (void)hipFree(tst);
  }
  if ((st = set_items(p, best_c))) { free_plan(p); return st; }
  p->tuned_ms = best;
  if (o.profile) {
    if ((err = hipEventCreate(&p->ev0)) != hipSuccess || (err = hipEventCreate(&p->ev1)) != hipSuccess) {
      free_plan(p);
      return api_hip_fail(err, "profiling events");
    }
    p->profile = true;
  }
  p->workspace_bytes = total + (int64_t)(p->items_cap * (sizeof(Item) + p->nacc * sizeof(double)));
  if (p->use_graph && (err = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking)) != hipSuccess) {
    free_plan(p);
    return api_hip_fail(err, "capture stream");
  }
  *out = p;
  return GWF_OK;
}

gwf_status gwf_plan_fisher(gwf_plan* p, double* fisher, double* snr, int32_t* status, double cond_max,
                           double* cov, double* sigma, double* cond, double* inv_err, void* stream) {
  if (!p) return api_fail(GWF_E_INVALID_ARG, "plan is NULL");
  if (!fisher || !snr || !status) return api_fail(GWF_E_INVALID_ARG, "fisher, snr and status are required");
  if (sigma && std::isnan(cond_max)) return api_fail(GWF_E_INVALID_ARG, "cond_max is NaN");
  if (!sigma && (cov || cond || inv_err))
    return api_fail(GWF_E_INVALID_ARG, "inversion outputs given without sigma");
  Outs o{fisher, snr, status, cond_max, cov, sigma, cond, inv_err};
  hipStream_t s = (hipStream_t)stream;
  if (!p->use_graph) return enqueue(p, o, s);
  const void* key[8] = {fisher, snr, status, cov, sigma, cond, inv_err, nullptr};
  if (!p->exec || std::memcmp(key, p->key, sizeof key) != 0 || (sigma && cond_max != p->key_cond)) {
    if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    hipError_t err = hipStreamBeginCapture(p->cap, hipStreamCaptureModeRelaxed);
    if (err != hipSuccess) return api_hip_fail(err, "graph capture begin");
    gwf_status st = enqueue(p, o, p->cap);
    hipGraph_t g = nullptr;
    err = hipStreamEndCapture(p->cap, &g);
    if (st) { if (g) (void)hipGraphDestroy(g); return st; }
    if (err != hipSuccess) return api_hip_fail(err, "graph capture end");
    err = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) { p->exec = nullptr; return api_hip_fail(err, "graph instantiate"); }
    std::memcpy(p->key, key, sizeof key);
    p->key_cond = cond_max;
  }
  hipError_t err = hipGraphLaunch(p->exec, s);
  if (err != hipSuccess) return api_hip_fail(err, "graph launch");
  return GWF_OK;
}

gwf_status gwf_plan_set_network(gwf_plan* p, const gwf_network* net) {
  if (!p) return api_fail(GWF_E_INVALID_ARG, "plan is NULL");
  NetDesc nd;
  gwf_status st = api_pack_network(net, nd);
  if (st) return st;
  if (nd.n_site > p->n_site_alloc)
    return api_fail(GWF_E_INVALID_ARG, "%d sites: the plan holds site constants for %d", nd.n_site, p->n_site_alloc);
  p->net = nd;
  p->tab = net_has_tables(nd);
  if (p->exec) {                    // the captured graph holds the old network
    (void)hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
  }
  return GWF_OK;
}

gwf_status gwf_plan_adjoint(gwf_plan* p, const double* gbar, const int32_t* status, double w_snr,
                            double w_fisher, double* grad_event, double* grad, void* stream) {
  if (!p) return api_fail(GWF_E_INVALID_ARG, "plan is NULL");
  if (!gbar || !grad_event || !grad) return api_fail(GWF_E_INVALID_ARG, "gbar, grad_event and grad are required");
  if (!std::isfinite(w_snr) || !std::isfinite(w_fisher))
    return api_fail(GWF_E_INVALID_ARG, "w_snr and w_fisher must be finite");
  if (p->mixed) return api_fail(GWF_E_UNSUPPORTED, "the adjoint has no mixed form (create the plan without GWF_MIXED)");
  hipStream_t s = (hipStream_t)stream;
  // the events' constants (the same set-up kernel as gwf_plan_fisher)
  SetupArgs sa{};
  sa.par = p->ev.par; sa.ld = p->ev.ld; sa.n = p->n;
  sa.fmin = p->grid.fmin; sa.fmax = p->grid.fmax; sa.npts = p->grid.npts; sa.npts_plan = p->npts_plan;
  sa.npts_max = 0x7fffffff;
  sa.ecc = p->ev.ecc; sa.fref = p->ev.f_ref_ecc;
  sa.net = p->net; sa.flags = p->flags; sa.evc = p->evc; sa.sic = p->sic; sa.status = nullptr;
  sa.active = p->ev.active;
  hipError_t err = hipSuccess;
  if (!p->aec) {                    // the first adjoint call allocates its constants
    int64_t dummy = 0;
    err = dev_alloc((char**)&p->aec, (size_t)p->n * adjoint_event_bytes(), dummy);
    if (err == hipSuccess)
      err = dev_alloc((char**)&p->asc, (size_t)p->n * p->n_site_alloc * adjoint_site_bytes(), dummy);
    if (err != hipSuccess) {
      (void)hipFree(p->aec);
      (void)hipFree(p->asc);
      p->aec = nullptr;
      p->asc = nullptr;
      return api_fail(GWF_E_NOMEM, "adjoint constants of %lld events", (long long)p->n);
    }
    p->workspace_bytes += (int64_t)((size_t)p->n * (adjoint_event_bytes() + p->n_site_alloc * adjoint_site_bytes()));
  }
  err = launch_setup(sa, s);
  if (err == hipSuccess) {
    AdjSetupArgs ua{};
    ua.par = p->ev.par; ua.ld = p->ev.ld; ua.n = p->n; ua.active = p->ev.active; ua.par_mask = p->ev.par_mask;
    ua.net = p->net; ua.gbar = gbar; ua.status = status; ua.evc = p->evc; ua.sic = p->sic;
    ua.aec = p->aec; ua.asc = p->asc;
    err = launch_adjoint_setup(ua, p->npi, s);
  }
  if (err == hipSuccess) {
    AdjItemsArgs aa{};
    aa.net = p->net; aa.evc = p->evc; aa.sic = p->sic; aa.aec = p->aec; aa.asc = p->asc;
    aa.items = p->items; aa.n_items = p->n_items; aa.partial = p->partial;
    err = launch_adjoint_items(aa, p->npi, p->rot, s);
  }
  if (err == hipSuccess) {
    AdjCombineArgs ca{};
    ca.n = p->n; ca.n_site = p->net.n_site; ca.item_first = p->item_first; ca.partial = p->partial;
    ca.w_snr = w_snr; ca.w_fisher = w_fisher; ca.grad_event = grad_event; ca.grad = grad;
    err = launch_adjoint_combine(ca, s);
  }
  if (err != hipSuccess) return api_hip_fail(err, "plan adjoint launch");
  return GWF_OK;
}

gwf_status gwf_plan_get_info(const gwf_plan* p, gwf_plan_info* info) {
  if (!p || !info) return api_fail(GWF_E_INVALID_ARG, "plan or info is NULL");
  info->chunk = p->chunk;
  info->n_items = p->n_items;
  info->pad = 0;
  info->use_graph = p->use_graph ? 1 : 0;
  info->workspace_bytes = p->workspace_bytes;
  info->tuned_ms = p->tuned_ms;
  info->items_ms = 0.0;
  if (p->profile) {
    float ms = 0.0f;
    hipError_t err = hipEventSynchronize(p->ev1);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, p->ev0, p->ev1);
    if (err != hipSuccess) return api_hip_fail(err, "items-kernel timing");
    info->items_ms = ms;
  }
  return GWF_OK;
}

gwf_status gwf_plan_destroy(gwf_plan* p) {
  free_plan(p);
  return GWF_OK;
}

}  // extern "C"

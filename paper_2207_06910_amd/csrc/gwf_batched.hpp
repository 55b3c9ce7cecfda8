// gwf_batched.hpp -- argument blocks and launchers of the batched form.
#pragma once

#include "gwf_kernels.hpp"

namespace gwf {

struct Item {
  int32_t e, k0, k1;        // event, grid-point range [k0, k1)
  int32_t slot;             // partial-sum slot: the item's position in event order
};

struct SetupArgs {
  const double* par;
  int64_t ld, n;
  const double* ecc;          // [n] or NULL: e0 (with kFlagEcc)
  const double* fref;         // [n] or NULL: reference frequency of e0
  const double* fmin;
  const double* fmax;
  const int32_t* npts;
  const int32_t* npts_plan;   // grid lengths the items were built from
  int32_t npts_max;           // longer grids are flagged invalid (their items were
                              // sized as for a two-point grid)
  const uint8_t* active;      // [n_ifo][ld] or NULL: interferometers taking part
  NetDesc net;
  uint32_t flags;
  EventC* evc;                // [n]
  SiteC* sic;                 // [n][n_site]
  int32_t* status;            // [n] or NULL, output: parameter status of each event
};

struct ItemsArgs {
  const EventC* evc;
  const SiteC* sic;
  int32_t n_site;
  const Item* items;          // one workgroup per item, in this order
  int32_t n_items;
  const int32_t* n_items_dev; // NULL, or the item count in device memory (read in place of n_items)
  double* partial;            // [n_items][NACC]
  int64_t base;               // first item of the launch (set by the launcher)
};

struct CombineArgs {
  int64_t n;
  const EventC* evc;
  const int32_t* item_first;  // [n+1]: items of event e are item_first[e] .. item_first[e+1]-1
  const double* partial;
  double* fisher;             // [P][P][n]
  double* snr;                // [n]
  int32_t* status;            // [n]
  const uint32_t* par_mask;   // [n] or NULL: rows of each event's Fisher matrix (others 0)
  int64_t base;               // first (event, slot) pair of the launch (set by the launcher)
};

// The adjoint over work items (gwf_plan_adjoint).  AdjEventC and AdjSiteC
// are declared in gwf_adjoint.hpp.
struct AdjEventC;
struct AdjSiteC;

// One lane per event: the contractions of its Gbar and its sites' pattern
// derivatives, after the plan's set-up kernel (EventC, SiteC).
struct AdjSetupArgs {
  const double* par;          // [13][ld]: theta and psi of each event
  int64_t ld, n;
  const uint8_t* active;      // [n_ifo][ld] or NULL
  const uint32_t* par_mask;   // [n] or NULL
  NetDesc net;
  const double* gbar;         // [P][P][n]
  const int32_t* status;      // [n] or NULL: events with a nonzero status contribute zero
  const EventC* evc;
  const SiteC* sic;
  AdjEventC* aec;             // [n]
  AdjSiteC* asc;              // [n][n_site]
};

// One workgroup per item of the plan; the constants of the set-up kernels;
// each item's per-site sums written to its slot.
struct AdjItemsArgs {
  NetDesc net;
  const EventC* evc;
  const SiteC* sic;
  const AdjEventC* aec;
  const AdjSiteC* asc;
  const Item* items;          // one workgroup per item, in this order
  int32_t n_items;
  double* partial;            // [n_items][n_site][8]; NaN where the event is left out
  int64_t base;               // first item of the launch (set by the launcher)
};

struct AdjCombineArgs {
  int64_t n;
  int32_t n_site;
  const int32_t* item_first;  // [n+1]
  const double* partial;
  double w_snr, w_fisher;
  double* grad_event;         // [n][n_site][4]
  double* grad;               // [n_site][4]
};

hipError_t launch_adjoint_setup(const AdjSetupArgs& a, int npi, hipStream_t s);
hipError_t launch_adjoint_items(const AdjItemsArgs& a, int npi, bool rot, hipStream_t s);
// bytes of the adjoint's per-event and per-site constants
size_t adjoint_event_bytes();
size_t adjoint_site_bytes();
hipError_t launch_adjoint_combine(const AdjCombineArgs& a, hipStream_t s);

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// Work items built on the device: each event's count of items of at most
// `chunk` points (a grid outside 2..npts_max counts as two points), their
// exclusive prefix sum first[0..n] and the total in *n_items (one
// workgroup), then the items themselves, in slot order.
hipError_t launch_items_build(const int32_t* npts, int64_t n, int32_t chunk, int32_t npts_max, int32_t* first,
                              int32_t* n_items, Item* items, hipStream_t s);
hipError_t launch_setup(const SetupArgs& a, hipStream_t s);
// npi: phase-only parameters, 3 + 2 (tides) + 1 (eccentricity)
// tab: a site has a sampled noise curve; n_wg: the number of items (or a bound)
hipError_t launch_items(const ItemsArgs& a, int npi, bool rot, bool mixed, bool tab, int64_t n_wg, hipStream_t s);
hipError_t launch_combine(const CombineArgs& a, int npi, hipStream_t s);
int fisher_nacc(int npi);
int fisher_block();

}  // namespace gwf

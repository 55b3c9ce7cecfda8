// gwf_api_internal.hpp -- host helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/gwf.h"
#include "gwf_model.hpp"

// Record a formatted message for gwf_last_error() and return code.
gwf_status api_fail(gwf_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
gwf_status api_hip_fail(hipError_t err, const char* where);
// Validate a network and pack it into the kernels' by-value descriptor.
gwf_status api_pack_network(const gwf_network* net, gwf::NetDesc& nd);
// Checks shared by every call taking events and a grid.
gwf_status api_check_common(const gwf_events* ev, const gwf_grid* grid, uint32_t flags);
// Phase-only Fisher parameters of a call: 3, plus 2 with GWF_TIDAL, plus 1
// with GWF_ECCENTRIC (P = 8 + this).
inline int api_npi(uint32_t flags) {
  return 3 + ((flags & GWF_TIDAL) ? 2 : 0) + ((flags & GWF_ECCENTRIC) ? 1 : 0);
}

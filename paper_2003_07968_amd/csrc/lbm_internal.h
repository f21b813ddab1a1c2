// Library-internal entry points shared by the host runtime (lbm.hip) and the
// serving loop (server.cpp).  Not part of the C ABI: hidden from the shared
// library's exports.
#pragma once

#include "lbm.h"

namespace lbm_internal {

// lbm_moments for the density alone (FP64, [ny][nx], device), enqueued on the
// lattice's stream without waiting and without reading the sticky error.
__attribute__((visibility("hidden"))) lbm_status enqueue_density(lbm_handle *h, double *d_rho);

// lbm_get_populations (FP64, [9][ny][nx], device), enqueued on the lattice's
// stream without waiting.
__attribute__((visibility("hidden"))) lbm_status enqueue_populations(lbm_handle *h,
                                                                     double *d_f);

}  // namespace lbm_internal

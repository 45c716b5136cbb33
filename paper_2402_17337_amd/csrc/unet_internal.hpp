// unet_internal.hpp -- what the solver library needs to run a warm-start
// network it has been handed (same shared library, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "ibm_unet.h"

namespace ibm {
namespace unet {

hipStream_t net_stream(const ibm_unet* net);
void net_shape(const ibm_unet* net, int* max_batch, int* h, int* w);

}  // namespace unet
}  // namespace ibm

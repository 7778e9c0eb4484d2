// host_common.hpp -- host-side helpers shared by the library's entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "automat.h"
#include "msgsm.hpp"

namespace automat {

// Validate an automat_params table and convert it to the kernels' layout.
int32_t copy_params(const automat_params *params, MSGSM::Phase *dst, int32_t *n_phases);

// Compute-unit count of the current device (cached per device).
int32_t device_cus(int *cus);

}  // namespace automat

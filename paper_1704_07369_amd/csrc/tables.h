// Plan tables filled on the device from the spec of build_spec.
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace efm {

// Fills d_g64 (2 J n doubles) and, when d_g32 is set, its FP32 copy; blocks
// until the fill is done.  Returns the first HIP error.
hipError_t fill_tables_device(const TableSpec& S, double* d_g64, float* d_g32);

}  // namespace efm

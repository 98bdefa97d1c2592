// Launch interface of the split-BF16 MFMA x pass.
#pragma once

#include <hip/hip_runtime.h>

namespace efm {

// W, Z, G hold FP32 complex values (layouts as in kernels.hip); N = 16 or 32.
hipError_t launch_pencil_bf16(const void* W, const void* G, int J, int ncells, void* Z, int N,
                              hipStream_t st);

}  // namespace efm

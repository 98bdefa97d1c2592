// 3D operator on grids of N = 64, 128 (FP64) through LDS line FFTs along every
// axis, one term at a time through device memory.
#pragma once

#include "kernels.h"

namespace efm {

bool large3d_supported(int N);

// One pass over a.ncells cells of a 3D plan: a.W holds ncells x N^3 complex
// (the spectrum), a.Z ncells x N^3 complex (the term volume) followed by
// ncells x N^3 doubles (the FP64 accumulator); twiddles = exp(2 pi i j / N),
// j < N (FP64 pairs, device).  Events a.ev, when set: before the forward
// transform, after it, after the last term, after the final transpose.
hipError_t launch_large3d(const ChunkArgs& a, const void* twiddles, hipStream_t st);

}  // namespace efm

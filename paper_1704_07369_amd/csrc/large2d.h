// 2D operator on large grids (N = 64, 128, 256, 512; FP64) through LDS line FFTs.
#pragma once

#include "kernels.h"

namespace efm {

bool large2d_supported(int N);

// One pass over a.ncells cells of a 2D plan: a.W holds ncells x N^2 complex,
// a.Z ncells x J x N^2 complex; twiddles = exp(2 pi i j / N), j < N (FP64
// pairs, device).  Events a.ev, when set: before the forward rows, after the
// forward columns, after the per-term column pass, after the row pass.
hipError_t launch_large2d(const ChunkArgs& a, const void* twiddles, hipStream_t st);

}  // namespace efm

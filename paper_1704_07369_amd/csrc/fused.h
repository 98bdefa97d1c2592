// Fused schedule of the 3D operator: forward transform, then one kernel that
// runs every term's inverse transform on chip and accumulates the gain in
// FP64 registers (no per-term intermediates in device memory).
#pragma once

#include "kernels.h"

namespace efm {

// x split P of the fused kernel (each cell is handled by P workgroups, one per
// residue class of the output x index mod P): the default for (N, precision),
// or 0 when the fused schedule has no instantiation for N.
int fused_default_split(int N, int precision);
bool fused_supported(int N, int precision, int split);

// The unnormalised 3D spectrum of every cell into a.W, half-space layout
// W[cell][kx][k2 < N/2][k1] (k_fwd3, or for small batches k_fwd and the
// in-place x pass k_fwdx), then k_fused.  Events a.ev, when set: before the
// forward transform, after it (twice), after k_fused.
hipError_t launch_fused(const ChunkArgs& a, int split, hipStream_t st);

// Term-parallel variant for small batches (3D, N = 16, 24, 32, FP64 or FP32,
// the splits of launch_fused): the forward transform into a.W as for
// launch_fused, then one workgroup per (cell, term, x residue) of the column
// (N = 32) or LDS-volume kernel writing its term's products to a.Z
// (ncells x J x N^3 doubles), then their sum per point into Q.  Events as for
// launch_fused (a.ev[3] after the sum).
bool terms_supported(int N, int precision, int split);
hipError_t launch_terms(const ChunkArgs& a, int split, hipStream_t st);

}  // namespace efm

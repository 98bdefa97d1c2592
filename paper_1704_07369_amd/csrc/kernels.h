// Internal launch interface of the HIP kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace efm {

// One pass of the collision pipeline over `ncells` consecutive cells of one
// plan: forward transform -> per-term multiply and inverse x transform ->
// per-term inverse slab transform with FP64 gain accumulation, loss and
// combine.  dt == 0 writes Q; dt != 0 writes Q = F + dt Q^s[F] (Q may equal f).
struct ChunkArgs {
  int N = 0, d = 0, precision = 0;
  int J = 0;                       // products + 1 (loss)
  const void* gamma = nullptr;     // [J][n] complex (FP64 or FP32 pairs)
  void* W = nullptr;               // workspace [ncells][n] complex
  void* Z = nullptr;               // workspace [ncells][J][n] complex (3D only)
  const double* f = nullptr;
  double* Q = nullptr;
  const int64_t* off = nullptr;    // device: element offset of every batch cell
  int64_t cell0 = 0;               // first batch cell of the pass
  int ncells = 0;
  double dt = 0.0;
  const void* tw = nullptr;        // 2D grids of N >= 64: exp(2 pi i j / N) table
  // optional: 4 events recorded before k_fwd, after k_fwd, after the x pass
  // and after k_slab (profiling; all on the launch stream)
  hipEvent_t* ev = nullptr;
};

hipError_t launch_chunk(const ChunkArgs& a, hipStream_t s);

// Q = sum of the term partials a.Z ([ncells][J][n] doubles) per point in the
// fused kernel's order (the loss term's -F l first, then the terms); Euler
// update when a.dt != 0.  Records a.ev[3] after it when a.ev is set.
hipError_t launch_terms_reduce(const ChunkArgs& a, int n, hipStream_t s);

// 2D term-parallel schedule (N = 8, 12, 16, 24, 32; FP64 or FP32): the
// forward transform into a.W, one block per (cell, term) writing that term's
// products to a.Z (ncells x J x N^2 doubles), then launch_terms_reduce.
bool terms_2d_supported(int N);
hipError_t launch_terms_2d(const ChunkArgs& a, hipStream_t s);

// k_fwd alone (3D, N = 16, 24, 32) into the half-space layout
// W[cell][x][k2 < N/2][k1]: the 2D transform of every x slab.  No events.
hipError_t launch_fwd_half_slabs(const ChunkArgs& a, hipStream_t s);

// Per-cell reductions (fixed order, deterministic).  Any output may be null.
//   full:    [cell][EC_NMON]
//   entprod: [cell]      n_nonpos: [cell]
//   step_mon: (mass, eta) at [(*step) * step_stride + cell][2]; step and the
//             capacity step_cap are read on device; nothing is written once
//             *step >= *step_cap
// cell_geo: (N, d) per cell; cell_L: L per cell (the grid points of the
// momentum and energy of Q, written to full[c * 11 + 7 .. 10] when Q is given)
hipError_t launch_monitors(const double* f, const double* Q, const int64_t* off,
                           const int* cell_n, const double* cell_hd, const int* cell_geo,
                           const double* cell_L, int64_t cell0, int64_t ncells, double* full,
                           double* entprod, int32_t* n_nonpos, const int* step,
                           double* step_mon, int64_t step_stride, const int* step_cap,
                           hipStream_t s);

hipError_t launch_copy(const double* a, double* b, int64_t n, hipStream_t s);
// blocks x 256 threads, each valu_probe_chains() FMA chains of iters steps;
// precision 0: FP64, 1: FP32; sink: one element of device memory
hipError_t launch_valu_probe(int precision, int blocks, int iters, void* sink, hipStream_t s);
int valu_probe_chains();
// out = a x + b y over the n points of each of the first ncells cells
hipError_t launch_axpby_cells(const double* x, const double* y, double* out, double a, double b,
                              const int64_t* off, const int* cell_n, int64_t ncells,
                              hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
hipError_t launch_inc_int(int* p, hipStream_t s);

}  // namespace efm

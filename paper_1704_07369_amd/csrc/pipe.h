// Launch interface of the software-pipelined 3D collision kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace efm {

// One launch: four roles on four chunks of one plan.  A role with n == 0 is
// absent.  Ring slots alternate between consecutive launches.
struct PipeArgs {
  const void* gamma = nullptr;    // [J][n] complex (precision of the kernel)
  int J = 0;                      // products + 1 (loss)
  int G = 1;                      // term groups of the P and S roles
  int chunk = 1;                  // cells per full chunk (ring stride)
  const double* f = nullptr;
  double* Q = nullptr;
  const int64_t* off = nullptr;
  double dt = 0.0;
  void* W[2] = {nullptr, nullptr};      // [chunk][n] complex
  void* Z[2] = {nullptr, nullptr};      // [chunk][J][n] complex
  double* Pg[2] = {nullptr, nullptr};   // [G][chunk][n]
  double* Lr[2] = {nullptr, nullptr};   // [chunk][n]
  int64_t f_cell0 = 0, p_cell0 = 0, s_cell0 = 0, c_cell0 = 0;
  int f_n = 0, p_n = 0, s_n = 0, c_n = 0;
  int f_slot = 0, p_slot = 0, s_slot = 0, c_slot = 0;
  int f_blocks = 0, p_blocks = 0, s_blocks = 0, c_blocks = 0;   // filled by launch
};

hipError_t launch_pipe(PipeArgs& a, int N, int precision, hipStream_t s);

}  // namespace efm

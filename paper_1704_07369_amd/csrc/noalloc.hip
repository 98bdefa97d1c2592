// ec_collide_noalloc: the collision operator of contiguous 3D cells on the
// fused schedule with no device allocation.  Its device memory beyond f and
// Q (the half-space spectra of one pass of cells and their offsets) is one
// fixed array, `scratch`, that the code object carries; each device holds its
// own copy, located once per device with hipGetSymbolAddress.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <exception>
#include <mutex>
#include <new>

#include "../../include/ec.h"
#include "fused.h"
#include "internal.h"

using namespace efm;

namespace {

// Pass-wide scratch: [kOffBytes] cell offsets, then the half-space spectra.
__device__ __align__(256) unsigned char scratch[EC_NOALLOC_SCRATCH_BYTES];

constexpr int64_t kOffCells = 8192;                   // most cells in one pass
constexpr int64_t kOffBytes = kOffCells * sizeof(int64_t);
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};                     // device address of scratch, per device

__global__ __launch_bounds__(256) void k_cell_offsets(int64_t* __restrict__ off, int64_t n,
                                                      int64_t stride) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) off[i] = i * stride;
}

// The device address of this device's scratch (the array's name is only a
// host-side handle; kernels must receive this address).
int scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(EC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
    }
    g_scratch[dev] = p;
  }
  *out = (unsigned char*)g_scratch[dev];
  return EC_OK;
}

int collide_noalloc(const ec_plan* plan, int precision, int64_t n_cells, const double* f,
                    double* Q, hipStream_t st) {
  if (!plan || !f || !Q) return set_error(EC_ERR_ARG, "null argument");
  if ((const void*)f == (const void*)Q) return set_error(EC_ERR_ARG, "f and Q must not alias");
  if (n_cells < 0) return set_error(EC_ERR_ARG, "n_cells < 0");
  if (precision != EC_FP64 && precision != EC_FP32)
    return set_error(EC_ERR_ARG, "precision must be EC_FP64 or EC_FP32");
  const int N = plan_N(plan);
  if (plan_d(plan) != 3 || fused_default_split(N, precision) == 0)
    return set_error(EC_ERR_UNSUPPORTED,
                     "ec_collide_noalloc needs 3D cells of N = 16, 24 or 32 (the fused schedule)");
  const void* gamma = plan_gamma(plan, precision);
  if (!gamma) return set_error(EC_ERR_UNSUPPORTED, "the plan keeps no tables in this precision");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_error(EC_ERR_DEVICE, "no HIP device");
  if (dev != plan_device(plan))
    return set_error(EC_ERR_ARG, "the plan was set up on another device than the current one");
  if (dev < 0 || dev >= kMaxDevices) return set_error(EC_ERR_UNSUPPORTED, "device index >= 64");
  const int64_t n = (int64_t)N * N * N;
  const int64_t per_cell = n / 2 * (precision == EC_FP64 ? 16 : 8);   // half-space spectrum
  const int64_t cap = std::min<int64_t>(
      kOffCells, ((int64_t)EC_NOALLOC_SCRATCH_BYTES - kOffBytes) / per_cell);
  if (cap < 1)
    return set_error(EC_ERR_UNSUPPORTED, "one cell's spectrum exceeds the scratch size");
  if (n_cells == 0) return EC_OK;
  unsigned char* base = nullptr;
  int rc = scratch_address(dev, &base);
  if (rc) return rc;
  int64_t* off = (int64_t*)base;
  void* W = base + kOffBytes;
  const int64_t first = std::min(cap, n_cells);
  hipLaunchKernelGGL(k_cell_offsets, dim3((unsigned)((first + 255) / 256)), dim3(256), 0, st, off,
                     first, n);
  hipError_t e = hipGetLastError();
  for (int64_t c0 = 0; c0 < n_cells && e == hipSuccess; c0 += cap) {
    ChunkArgs a;
    a.N = N; a.d = 3; a.precision = precision; a.J = plan_J(plan);
    a.gamma = gamma;
    a.W = W;
    a.f = f + c0 * n;
    a.Q = Q + c0 * n;
    a.off = off;
    a.cell0 = 0;
    a.ncells = (int)std::min(cap, n_cells - c0);
    a.dt = 0.0;
    e = launch_fused(a, fused_split_for_cells(N, precision, a.ncells), st);
  }
  if (e != hipSuccess) return set_error(EC_ERR_DEVICE, hipGetErrorString(e));
  return EC_OK;
}

}  // namespace

extern "C" int ec_collide_noalloc(const ec_plan* plan, int precision, int64_t n_cells,
                                  const double* f, double* Q, void* hip_stream) {
  try {
    return collide_noalloc(plan, precision, n_cells, f, Q, (hipStream_t)hip_stream);
  } catch (const std::bad_alloc&) {
    return set_error(EC_ERR_OOM, "host allocation failed");
  } catch (const std::exception& ex) {
    return set_error(EC_ERR_ARG, ex.what());
  }
}

// Plan tables filled on the device: one thread per mode evaluates the same
// per-mode formulas as the host fill (table_math.h) and writes the FP64
// table and, when requested, its FP32 copy.
#include "tables.h"

#include "table_math.h"

namespace efm {

__global__ __launch_bounds__(256) void k_fill_tables(TableView V, double* __restrict__ g64,
                                                     float* __restrict__ g32) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= V.n) return;
  fill_mode(V, idx, g64, g32);
}

hipError_t fill_tables_device(const TableSpec& S, double* d_g64, float* d_g32) {
  // the spec arrays, packed into one upload
  std::vector<double> dbl;
  auto put = [&](const std::vector<double>& v) {
    const size_t o = dbl.size();
    dbl.insert(dbl.end(), v.begin(), v.end());
    return o;
  };
  const size_t o_ex = put(S.ex), o_ey = put(S.ey), o_ez = put(S.ez), o_px = put(S.px),
               o_py = put(S.py), o_wt = put(S.wt), o_rho = put(S.rho), o_om = put(S.om),
               o_cheb = put(S.cheb), o_sig = put(S.sig1);
  double* d_dbl = nullptr;
  int* d_off = nullptr;
  hipError_t e = hipMalloc(&d_dbl, std::max<size_t>(1, dbl.size()) * sizeof(double));
  if (e != hipSuccess) return e;
  e = hipMalloc(&d_off, std::max<size_t>(1, S.cheb_off.size()) * sizeof(int));
  if (e == hipSuccess && !dbl.empty())
    e = hipMemcpy(d_dbl, dbl.data(), dbl.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess && !S.cheb_off.empty())
    e = hipMemcpy(d_off, S.cheb_off.data(), S.cheb_off.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    TableView V;
    V.N = S.N; V.d = S.d; V.M = S.M; V.nrad = S.nrad; V.radial = S.radial ? 1 : 0;
    V.n = S.n; V.J = S.J; V.R = S.R; V.kf = S.kf; V.scale = S.scale; V.qmax = S.qmax;
    V.ex = d_dbl + o_ex; V.ey = d_dbl + o_ey; V.ez = d_dbl + o_ez;
    V.px = d_dbl + o_px; V.py = d_dbl + o_py; V.wt = d_dbl + o_wt;
    V.rho = d_dbl + o_rho; V.om = d_dbl + o_om;
    V.cheb = d_dbl + o_cheb; V.cheb_off = d_off; V.sig1 = d_dbl + o_sig;
    hipLaunchKernelGGL(k_fill_tables, dim3((unsigned)((S.n + 255) / 256)), dim3(256), 0, 0, V,
                       d_g64, d_g32);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  (void)hipFree(d_dbl);
  if (d_off) (void)hipFree(d_off);
  return e;
}

}  // namespace efm

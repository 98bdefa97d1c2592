// Per-mode formulas of the plan tables (the closed forms and Chebyshev fits
// documented in plan.cpp), host + device: the host fills the tables for
// ec_host_tables, the device fills them for a plan (csrc/tables.hip).  One
// call writes every table entry of one mode, so modes are independent.
#pragma once

#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define TM_HD __host__ __device__ __forceinline__
#else
#define TM_HD inline
#endif

namespace efm {

// Everything the per-mode fill reads (plain pointers: host or device arrays).
struct TableView {
  int N = 0, d = 0, M = 0, nrad = 1, radial = 0;
  int64_t n = 0;          // points (modes) per cell
  int J = 0;              // table entries per mode: M nrad products + the loss
  double R = 0, kf = 0, scale = 0, qmax = 0;
  const double* ex = nullptr;     // directions (M)
  const double* ey = nullptr;
  const double* ez = nullptr;
  const double* px = nullptr;     // 2D partner directions (M)
  const double* py = nullptr;
  const double* wt = nullptr;     // direction weights (M)
  const double* rho = nullptr;    // radial nodes and weights (nrad)
  const double* om = nullptr;
  const double* cheb = nullptr;   // Chebyshev coefficients of Phi_j on [0, qmax]
  const int* cheb_off = nullptr;  // nrad + 1 offsets into cheb
  const double* sig1 = nullptr;   // 1D filter (N)
};

TM_HD double tm_sinc(double x) {
  if (fabs(x) < 1e-4) {
    const double x2 = x * x;
    return 1.0 - x2 / 6.0 + x2 * x2 / 120.0;
  }
  return sin(x) / x;
}

// 2D: int_{-R}^{R} cos(rho s) d rho
TM_HD double tm_psi2(double s, double R) { return 2.0 * R * tm_sinc(R * s); }

// 3D: int_{-R}^{R} |rho| cos(rho s) d rho
TM_HD double tm_psi3(double s, double R) {
  const double x = R * s;
  const double h = tm_sinc(0.5 * x);
  return 2.0 * R * R * (tm_sinc(x) - 0.5 * h * h);
}

// 3D: 2 int_{disk R} cos(k.x) dx = 4 pi R^2 J_1(R q) / (R q)
TM_HD double tm_phi3(double q, double R) {
  const double PI_ = 3.14159265358979323846;
  const double x = R * q;
  double j1x;
  if (x < 1e-4) {
    j1x = 0.5 - x * x / 16.0;
  } else {
#if defined(__HIP_DEVICE_COMPILE__)
    j1x = j1(x) / x;
#else
    j1x = std::cyl_bessel_j(1.0, x) / x;
#endif
  }
  return 4.0 * PI_ * R * R * j1x;
}

// Clenshaw sum of a Chebyshev series on [0, qmax]
TM_HD double tm_cheb(const double* c, int D, double qmax, double q) {
  const double x = qmax > 0.0 ? 2.0 * q / qmax - 1.0 : -1.0;
  double b1 = 0.0, b2 = 0.0;
  for (int k = D - 1; k >= 1; --k) {
    const double b0 = 2.0 * x * b1 - b2 + c[k];
    b2 = b1;
    b1 = b0;
  }
  return x * b1 - b2 + c[0];
}

// All J entries of mode idx = ((i0 n2 + i2) n1 + i1) (2D: i0 = 0):
// g64[(term out_n + out_idx) * 2 + {0, 1}] and, when g32 is set, its FP32
// copy.  The full table is out_n = n, out_idx = idx (fill_mode).
TM_HD void fill_mode_at(const TableView& V, int64_t idx, int64_t out_n, int64_t out_idx,
                        double* g64, float* g32) {
  const int N = V.N;
  auto mode = [N](int i) { return i < (N + 1) / 2 ? i : i - N; };
  int i0 = 0, i1, i2;
  if (V.d == 3) {
    i0 = (int)(idx / ((int64_t)N * N));
    i2 = (int)((idx / N) % N);
    i1 = (int)(idx % N);
  } else {
    i2 = (int)(idx / N);
    i1 = (int)(idx % N);
  }
  double kx, ky, kz, sig;
  if (V.d == 3) {
    kx = mode(i0); ky = mode(i1); kz = mode(i2);
    sig = V.sig1[i0] * V.sig1[i1] * V.sig1[i2];
  } else {
    kx = mode(i1); ky = mode(i2); kz = 0.0;
    sig = V.sig1[i1] * V.sig1[i2];
  }
  auto put = [&](int64_t term, double re, double im) {
    const int64_t e = (term * out_n + out_idx) * 2;
    g64[e] = re;
    g64[e + 1] = im;
    if (g32) {
      g32[e] = (float)re;
      g32[e + 1] = (float)im;
    }
  };
  const double k2 = kx * kx + ky * ky + kz * kz;
  const double kf = V.kf, scale = V.scale;
  double diag = 0.0;
  for (int t = 0; t < V.M; ++t) {
    const double kd = kx * V.ex[t] + ky * V.ey[t] + kz * V.ez[t];
    if (V.radial) {
      const double q = kf * sqrt(fmax(0.0, k2 - kd * kd));
      for (int j = 0; j < V.nrad; ++j) {
        const double ps = 2.0 * V.om[j] * V.rho[j] * cos(V.rho[j] * kf * kd);
        const double ph = tm_cheb(V.cheb + V.cheb_off[j], V.cheb_off[j + 1] - V.cheb_off[j],
                                  V.qmax, q);
        put((int64_t)t * V.nrad + j, scale * V.wt[t] * sig * ps, scale * sig * ph);
        diag += V.wt[t] * ps * ph;
      }
      continue;
    }
    double ps, ph;
    if (V.d == 2) {
      ps = tm_psi2(kf * kd, V.R);
      ph = tm_psi2(kf * (kx * V.px[t] + ky * V.py[t]), V.R);
    } else {
      ps = tm_psi3(kf * kd, V.R);
      ph = tm_phi3(kf * sqrt(fmax(0.0, k2 - kd * kd)), V.R);
    }
    put(t, scale * V.wt[t] * sig * ps, scale * sig * ph);
    diag += V.wt[t] * ps * ph;
  }
  put((int64_t)V.J - 1, scale * sig * sig * diag, 0.0);
}

TM_HD void fill_mode(const TableView& V, int64_t idx, double* g64, float* g32) {
  fill_mode_at(V, idx, V.n, idx, g64, g32);
}

}  // namespace efm

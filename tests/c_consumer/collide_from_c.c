/*
 * A C program on the library's C ABI alone (no Python, no torch): a 3D
 * hard-sphere plan (N = 16, M = 8, L = 8, R = 6), a batch of two cells
 * (F = 0 and an anisotropic Gaussian), Q on the device, and two checks on the
 * host: Q = 0 exactly for F = 0, and |sum Q| <= 1e-13 sum |Q| for the
 * Gaussian (the discrete mass conservation of Theorem 1).  Prints "ok" and
 * returns 0 on success; prints what failed and returns 1 otherwise.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "ec.h"

static int fail(const char* what) {
  fprintf(stderr, "%s failed: %s\n", what, ec_last_error());
  return 1;
}

int main(void) {
  const int N = 16, d = 3, M = 8;
  const double L = 8.0, pi = 3.14159265358979323846;
  ec_kernel k;
  memset(&k, 0, sizeof k);
  k.kind = EC_KERNEL_HARD_SPHERE;
  k.R = 6.0;
  ec_plan* plan = NULL;
  if (ec_setup_kernel(N, d, L, &k, M, &plan) != 0) return fail("ec_setup_kernel");
  const ec_plan* plans[1] = {plan};
  const int64_t counts[1] = {2};
  ec_batch* b = NULL;
  if (ec_batch_create(plans, counts, 1, EC_FP64, &b) != 0) return fail("ec_batch_create");
  int64_t ncell = 0, nel = 0, off[2];
  if (ec_batch_size(b, &ncell, &nel) != 0 || ncell != 2) return fail("ec_batch_size");
  if (ec_batch_offsets(b, off) != 0) return fail("ec_batch_offsets");

  double* hf = (double*)calloc((size_t)nel, sizeof(double));
  double* hq = (double*)calloc((size_t)nel, sizeof(double));
  if (!hf || !hq) return 1;
  const double h = 2.0 * L / N;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int l = 0; l < N; ++l) {
        const double vx = -L + i * h - 0.5, vy = -L + j * h + 0.25, vz = -L + l * h;
        hf[off[1] + ((int64_t)i * N + j) * N + l] =
            exp(-0.5 * (vx * vx / 1.2 + vy * vy / 0.8 + vz * vz)) / pow(2.0 * pi, 1.5);
      }
  double *df = NULL, *dq = NULL;
  if (hipMalloc((void**)&df, (size_t)nel * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&dq, (size_t)nel * sizeof(double)) != hipSuccess) {
    fprintf(stderr, "hipMalloc failed\n");
    return 1;
  }
  if (hipMemcpy(df, hf, (size_t)nel * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return 1;
  if (ec_collide(b, df, dq, NULL) != 0) return fail("ec_collide");
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(hq, dq, (size_t)nel * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
    fprintf(stderr, "device error\n");
    return 1;
  }

  const int64_t n = (int64_t)N * N * N;
  for (int64_t r = 0; r < n; ++r)
    if (hq[off[0] + r] != 0.0) {
      fprintf(stderr, "Q of the zero cell is %g at %lld\n", hq[off[0] + r], (long long)r);
      return 1;
    }
  double s = 0.0, sa = 0.0;
  for (int64_t r = 0; r < n; ++r) {
    s += hq[off[1] + r];
    sa += fabs(hq[off[1] + r]);
  }
  if (!(sa > 0.0) || fabs(s) > 1e-13 * sa) {
    fprintf(stderr, "mass: |sum Q| = %g, sum |Q| = %g\n", fabs(s), sa);
    return 1;
  }
  printf("|sum Q| / sum |Q| = %.3e\n", fabs(s) / sa);
  hipFree(df);
  hipFree(dq);
  free(hf);
  free(hq);
  if (ec_batch_destroy(b) != 0 || ec_plan_destroy(plan) != 0) return fail("destroy");
  printf("ok\n");
  return 0;
}

// In-register mixed-radix FFTs for one line of N complex values held by one
// thread.  Host+device so the same code is unit-tested on the CPU.
//
// Algorithm: Stockham autosort, decimation in frequency.  With the current
// sub-length n (starting at N), stride s (starting at 1) and radix R, m = n/R:
//   y[q + s (R p + u)] = w_n^{p u} * sum_r w_R^{r u} x[q + s (p + r m)]
// for p < m, q < s, u < R; then n <- m, s <- s R.  The output is in natural
// order.  w_n = exp(SIGN 2 pi i / n).  All indices are compile-time after
// unrolling, so the data stays in registers and the twiddles fold to
// immediates (trivial ones vanish).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define EFM_HD __host__ __device__ __forceinline__
#else
#define EFM_HD inline
#endif

#include "twiddles.h"

namespace efm {

template <typename R>
struct cx {
  R x, y;
};

template <typename R> EFM_HD cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> EFM_HD cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R> EFM_HD cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by SIGN*i
template <int SIGN, typename R> EFM_HD cx<R> mul_i(cx<R> a) {
  if constexpr (SIGN > 0) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// v * exp(SIGN 2 pi i j / N)
template <int N, int SIGN, typename R>
EFM_HD cx<R> twiddle(cx<R> v, int j) {
  j %= N;
  if (j == 0) return v;
  if (4 * j == N) return mul_i<SIGN>(v);
  if (2 * j == N) return {-v.x, -v.y};
  if (4 * j == 3 * N) return mul_i<-SIGN>(v);
  const R c = (R)Tw<N>::c[j];
  const R s = (R)(SIGN > 0 ? Tw<N>::s[j] : -Tw<N>::s[j]);
  return {v.x * c - v.y * s, v.x * s + v.y * c};
}

// a[u] <- sum_r a[r] w_R^{r u}
template <int RADIX, int SIGN, typename R>
EFM_HD void butterfly(cx<R> (&a)[RADIX]) {
  if constexpr (RADIX == 2) {
    cx<R> t0 = cadd(a[0], a[1]), t1 = csub(a[0], a[1]);
    a[0] = t0; a[1] = t1;
  } else if constexpr (RADIX == 4) {
    cx<R> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
    cx<R> s13 = cadd(a[1], a[3]), d13 = mul_i<SIGN>(csub(a[1], a[3]));
    a[0] = cadd(s02, s13); a[2] = csub(s02, s13);
    a[1] = cadd(d02, d13); a[3] = csub(d02, d13);
  } else if constexpr (RADIX == 3) {
    // w_3 = -1/2 + SIGN i sqrt(3)/2
    const R h = (R)0.5, r3 = (R)Tw<3>::s[1];
    cx<R> s = cadd(a[1], a[2]);
    cx<R> d = mul_i<SIGN>(csub(a[1], a[2]));
    cx<R> m = {a[0].x - h * s.x, a[0].y - h * s.y};
    a[0] = cadd(a[0], s);
    a[1] = {m.x + r3 * d.x, m.y + r3 * d.y};
    a[2] = {m.x - r3 * d.x, m.y - r3 * d.y};
  } else {
    static_assert(RADIX == 2 || RADIX == 3 || RADIX == 4, "radix");
  }
}

constexpr int pick_radix(int n) { return (n % 4 == 0) ? 4 : (n % 3 == 0 ? 3 : 2); }

template <int N, int n, int s, int SIGN, typename R>
EFM_HD void stockham_stage(cx<R> (&x)[N]) {
  if constexpr (n > 1) {
    constexpr int RADIX = pick_radix(n);
    constexpr int m = n / RADIX;
    cx<R> y[N];
#pragma unroll
    for (int p = 0; p < m; ++p) {
#pragma unroll
      for (int q = 0; q < s; ++q) {
        cx<R> a[RADIX];
#pragma unroll
        for (int r = 0; r < RADIX; ++r) a[r] = x[q + s * (p + r * m)];
        butterfly<RADIX, SIGN>(a);
#pragma unroll
        for (int u = 0; u < RADIX; ++u) y[q + s * (RADIX * p + u)] = twiddle<N, SIGN>(a[u], p * u * (N / n));
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = y[i];
    stockham_stage<N, m, s * RADIX, SIGN>(x);
  }
}

// In-place DFT of a register line: X[k] = sum_j x[j] exp(SIGN 2 pi i j k / N).
template <int N, int SIGN, typename R>
EFM_HD void fft_line(cx<R> (&x)[N]) {
  if constexpr (N > 1) stockham_stage<N, N, 1, SIGN>(x);
}

}  // namespace efm

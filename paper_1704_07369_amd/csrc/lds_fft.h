// Line FFTs in LDS for grids whose lines do not fit in registers (N = 64 ..
// 512, FP64): Stockham radix-4 stages (one radix-2 stage when log2 N is odd)
// over NL lines of N complex values stored contiguously, twiddles from a
// per-plan FP64 table tw[j] = exp(2 pi i j / N).
#pragma once

#include "fft.h"

namespace efm {

constexpr int L2D_BS = 256;
constexpr int COLS = 8;   // columns per workgroup of the column passes

template <int N>
constexpr int log4_stages() {
  int s = 0, n = N;
  while (n % 4 == 0) { n /= 4; ++s; }
  return s;
}

// Stockham stages over NL lines of length N stored contiguously in LDS
// (line l at x[l * N]); ping-pong between x and y; returns the buffer that
// holds the result.  SIGN: -1 forward, +1 inverse (unnormalised).
template <int N, int SIGN, int NL>
__device__ cx<double>* lds_fft(cx<double>* x, cx<double>* y, const cx<double>* __restrict__ tw) {
  constexpr int S4 = log4_stages<N>();
  int n = N, s = 1;
#pragma unroll
  for (int st = 0; st < S4; ++st) {
    const int m = n / 4;
    for (int b = threadIdx.x; b < NL * (N / 4); b += L2D_BS) {
      const int l = b / (N / 4), bb = b % (N / 4);
      const int p = bb / s, q = bb % s;
      const cx<double>* xl = x + l * N;
      cx<double>* yl = y + l * N;
      cx<double> a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = xl[q + s * (p + r * m)];
      butterfly<4, SIGN>(a);
      const int step = N / n;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = (p * u * step) % N;
        cx<double> w = tw[j];
        if (SIGN < 0) w.y = -w.y;
        yl[q + s * (4 * p + u)] = u == 0 ? a[0] : cmul(a[u], w);
      }
    }
    __syncthreads();
    cx<double>* t = x; x = y; y = t;
    n = m;
    s *= 4;
  }
  if constexpr ((N >> (2 * S4)) == 2) {
    // final radix-2 stage: n = 2, m = 1, p = 0 (no twiddles)
    for (int b = threadIdx.x; b < NL * (N / 2); b += L2D_BS) {
      const int l = b / (N / 2), q = b % (N / 2);
      const cx<double>* xl = x + l * N;
      cx<double>* yl = y + l * N;
      const cx<double> a0 = xl[q], a1 = xl[q + s];
      yl[q] = cadd(a0, a1);
      yl[q + s] = csub(a0, a1);
    }
    __syncthreads();
    cx<double>* t = x; x = y; y = t;
  }
  return x;
}

}  // namespace efm

// 2D operator on large grids (N = 64 .. 512) for gfx950.
//
// A line of N <= 512 complex FP64 values (8 KiB) is transformed in LDS by a
// Stockham radix-4 FFT (one radix-2 stage when log2 N is odd), with twiddles
// from a per-plan FP64 table tw[j] = exp(2 pi i j / N) (exactly reduced on the
// host).  One evaluation of a cell of N x N (F[y][z], z fastest):
//   k2_rows_fwd   rows: forward DFT along z          -> A[y][kz]
//   k2_cols_fwd   column groups of 8: forward along y -> A = Fh[ky][kz] in place
//   k2_cols_term  per term and column group: gamma_t Fh, inverse along y
//                                                    -> C[t][y][kz]
//   k2_rows_acc   rows: per term inverse along z, gain += Re c Im c (FP64),
//                 the last term gives the loss l; Q = gain - F l (or F + dt Q)
// Column groups of 8 complex FP64 values read and write 128-byte row
// segments.  Tables are gamma[t][kz][ky] (ky fastest), as for every 2D plan.
#include "large2d.h"

#include "fft.h"
#include "lds_fft.h"

namespace efm {

template <int N>
constexpr int rows_per_block() { return (4 * L2D_BS) / N >= 1 ? (4 * L2D_BS) / N : 1; }

// forward DFT along z of every row of F -> A[cell][y][kz]
template <int N>
__global__ __launch_bounds__(L2D_BS) void k2_rows_fwd(const double* __restrict__ f,
                                                      const int64_t* __restrict__ off,
                                                      int64_t cell0, int ncells,
                                                      const cx<double>* __restrict__ tw,
                                                      cx<double>* __restrict__ A) {
  constexpr int NL = rows_per_block<N>();
  __shared__ cx<double> b0[NL * N], b1[NL * N];
  const int64_t row0 = (int64_t)blockIdx.x * NL;
  const int64_t rows = (int64_t)ncells * N;
  for (int i = threadIdx.x; i < NL * N; i += L2D_BS) {
    const int64_t row = row0 + i / N;
    double v = 0.0;
    if (row < rows) v = f[off[cell0 + row / N] + (row % N) * N + i % N];
    b0[i] = {v, 0.0};
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, -1, NL>(b0, b1, tw);
  for (int i = threadIdx.x; i < NL * N; i += L2D_BS) {
    const int64_t row = row0 + i / N;
    if (row < rows) A[row * N + i % N] = r[i];
  }
}

// forward DFT along y of column groups of A, in place
template <int N>
__global__ __launch_bounds__(L2D_BS) void k2_cols_fwd(int ncells, const cx<double>* __restrict__ tw,
                                                      cx<double>* __restrict__ A) {
  __shared__ cx<double> b0[COLS * N], b1[COLS * N];
  const int64_t g = blockIdx.x;                // (cell, column group)
  const int64_t cc = g / (N / COLS);
  const int c0 = (int)(g % (N / COLS)) * COLS;
  if (cc >= ncells) return;
  cx<double>* Ac = A + cc * N * N;
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int y = i / COLS, c = i % COLS;        // coalesced: consecutive columns
    b0[c * N + y] = Ac[(int64_t)y * N + c0 + c];
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, -1, COLS>(b0, b1, tw);
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int y = i / COLS, c = i % COLS;
    Ac[(int64_t)y * N + c0 + c] = r[c * N + y];
  }
}

// per term: gamma_t Fh on a column group, inverse DFT along y -> C[cell][t][y][kz]
template <int N>
__global__ __launch_bounds__(L2D_BS) void k2_cols_term(int ncells, int J,
                                                       const cx<double>* __restrict__ G,
                                                       const cx<double>* __restrict__ tw,
                                                       const cx<double>* __restrict__ A,
                                                       cx<double>* __restrict__ C) {
  __shared__ cx<double> b0[COLS * N], b1[COLS * N];
  const int64_t g = blockIdx.x;                // (cell, term, column group)
  const int groups = N / COLS;
  const int64_t cc = g / ((int64_t)J * groups);
  const int t = (int)((g / groups) % J);
  const int c0 = (int)(g % groups) * COLS;
  if (cc >= ncells) return;
  const cx<double>* Ac = A + cc * N * N;
  const cx<double>* Gt = G + (int64_t)t * N * N;
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int y = i / COLS, c = i % COLS;
    b0[c * N + y] = Ac[(int64_t)y * N + c0 + c];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int c = i / N, ky = i % N;             // table line kz = c0 + c, contiguous in ky
    b0[i] = cmul(Gt[(int64_t)(c0 + c) * N + ky], b0[i]);
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, +1, COLS>(b0, b1, tw);
  cx<double>* Ct = C + (cc * J + t) * N * N;
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int y = i / COLS, c = i % COLS;
    Ct[(int64_t)y * N + c0 + c] = r[c * N + y];
  }
}

// rows: for every term inverse DFT along z, FP64 gain, loss, combine
template <int N>
__global__ __launch_bounds__(L2D_BS) void k2_rows_acc(int ncells, int J,
                                                      const cx<double>* __restrict__ tw,
                                                      const cx<double>* __restrict__ C,
                                                      const double* f, const int64_t* __restrict__ off,
                                                      int64_t cell0, double* Q, double dt) {
  constexpr int NL = rows_per_block<N>();
  constexpr int PER = (NL * N + L2D_BS - 1) / L2D_BS;   // points per thread
  __shared__ cx<double> b0[NL * N], b1[NL * N];
  const int64_t row0 = (int64_t)blockIdx.x * NL;
  const int64_t rows = (int64_t)ncells * N;
  double acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0;
  for (int t = 0; t < J; ++t) {
    for (int i = threadIdx.x; i < NL * N; i += L2D_BS) {
      const int64_t row = row0 + i / N;
      cx<double> v = {0.0, 0.0};
      if (row < rows) {
        const int64_t cc = row / N, y = row % N;
        v = C[((cc * J + t) * N + y) * N + i % N];
      }
      b0[i] = v;
    }
    __syncthreads();
    const cx<double>* r = lds_fft<N, +1, NL>(b0, b1, tw);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + k * L2D_BS;
      if (i < NL * N) {
        const cx<double> c = r[i];
        if (t + 1 < J) {
          acc[k] += c.x * c.y;
        } else {
          const int64_t row = row0 + i / N;
          if (row < rows) {
            const int64_t idx = off[cell0 + row / N] + (row % N) * N + i % N;
            const double fv = f[idx];
            const double q = acc[k] - fv * c.x;
            Q[idx] = dt == 0.0 ? q : fv + dt * q;
          }
        }
      }
    }
    __syncthreads();                  // r is b0 or b1: the next term overwrites both
  }
}

template <int N>
static hipError_t launch_t(const ChunkArgs& a, const cx<double>* tw, hipStream_t st) {
  constexpr int NL = rows_per_block<N>();
  cx<double>* A = (cx<double>*)a.W;
  cx<double>* C = (cx<double>*)a.Z;
  const cx<double>* G = (const cx<double>*)a.gamma;
  const int64_t rows = (int64_t)a.ncells * N;
  const unsigned rblocks = (unsigned)((rows + NL - 1) / NL);
  if (a.ev) (void)hipEventRecord(a.ev[0], st);
  hipLaunchKernelGGL((k2_rows_fwd<N>), dim3(rblocks), dim3(L2D_BS), 0, st, a.f, a.off, a.cell0,
                     a.ncells, tw, A);
  hipLaunchKernelGGL((k2_cols_fwd<N>), dim3((unsigned)((int64_t)a.ncells * (N / COLS))),
                     dim3(L2D_BS), 0, st, a.ncells, tw, A);
  if (a.ev) (void)hipEventRecord(a.ev[1], st);
  hipLaunchKernelGGL((k2_cols_term<N>),
                     dim3((unsigned)((int64_t)a.ncells * a.J * (N / COLS))), dim3(L2D_BS), 0, st,
                     a.ncells, a.J, G, tw, (const cx<double>*)A, C);
  if (a.ev) (void)hipEventRecord(a.ev[2], st);
  hipLaunchKernelGGL((k2_rows_acc<N>), dim3(rblocks), dim3(L2D_BS), 0, st, a.ncells, a.J, tw,
                     (const cx<double>*)C, a.f, a.off, a.cell0, a.Q, a.dt);
  if (a.ev) (void)hipEventRecord(a.ev[3], st);
  return hipGetLastError();
}

bool large2d_supported(int N) { return N == 64 || N == 128 || N == 256 || N == 512; }

hipError_t launch_large2d(const ChunkArgs& a, const void* twiddles, hipStream_t st) {
  if (a.ncells <= 0) return hipSuccess;
  if (a.d != 2 || a.precision != 0) return hipErrorInvalidValue;
  const cx<double>* tw = (const cx<double>*)twiddles;
  switch (a.N) {
    case 64: return launch_t<64>(a, tw, st);
    case 128: return launch_t<128>(a, tw, st);
    case 256: return launch_t<256>(a, tw, st);
    case 512: return launch_t<512>(a, tw, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace efm

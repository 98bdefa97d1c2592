// 3D operator on grids whose lines do not fit in registers (N = 64, 128;
// FP64), every axis by LDS line FFTs and every term through device memory.
//
// One pass over a set of cells (F[x][y][z], z fastest; spectra and term
// volumes [x][k2][k1], k1 fastest, as the plan tables):
//   k3_rows_fwd    rows (x, y): forward DFT along z       -> B[x][y][kz]
//   k3_ycols_fwd   per x slab, groups of 8 kz: forward DFT along y
//                                                        -> A[x][kz][ky]
//   k3_xcols       groups of 8 ky per (kz): forward DFT along x, in place
//                                                        -> A = Fh[k0][k2][k1]
//   per term t (the loss term D first, then the gain terms):
//     k3_xcols     gamma_t Fh, inverse DFT along x       -> C[x][k2][k1]
//     k3_zcols     per x slab, groups of 8 k1: inverse DFT along z, in place
//                                                        -> C[x][z][k1]
//     k3_rows_acc  rows (x, z): inverse DFT along y; the loss term sets
//                  ACC[x][z][y] = -F l, the gain terms add Re c Im c (FP64)
//   k3_final       Q[x][y][z] = ACC[x][z][y] (or F + dt Q), 32 x 32 LDS tiles
// B shares the memory of C.  Column groups of 8 complex FP64 values read and
// write 128-byte segments.  The transforms, tables and normalisation are
// those of the other schedules (section 4.1, eq. fastAlg; the loss of
// section 3.1.2), so the result is the same operator.
#include "large3d.h"

#include "fft.h"
#include "lds_fft.h"

namespace efm {

template <int N>
constexpr int rows3_per_block() { return (4 * L2D_BS) / N; }

// forward DFT along z of every (cell, x, y) row of F -> B[cell][x][y][kz]
template <int N>
__global__ __launch_bounds__(L2D_BS) void k3_rows_fwd(const double* __restrict__ f,
                                                      const int64_t* __restrict__ off,
                                                      int64_t cell0, int ncells,
                                                      const cx<double>* __restrict__ tw,
                                                      cx<double>* __restrict__ B) {
  constexpr int NL = rows3_per_block<N>();
  __shared__ cx<double> b0[NL * N], b1[NL * N];
  const int64_t row0 = (int64_t)blockIdx.x * NL;
  const int64_t rows = (int64_t)ncells * N * N;
  for (int i = threadIdx.x; i < NL * N; i += L2D_BS) {
    const int64_t row = row0 + i / N;
    double v = 0.0;
    if (row < rows) v = f[off[cell0 + row / (N * N)] + (row % (N * N)) * N + i % N];
    b0[i] = {v, 0.0};
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, -1, NL>(b0, b1, tw);
  for (int i = threadIdx.x; i < NL * N; i += L2D_BS) {
    const int64_t row = row0 + i / N;
    if (row < rows) B[row * N + i % N] = r[i];
  }
}

// per x slab and group of 8 kz: forward DFT along y, B[x][y][kz] -> A[x][kz][ky]
template <int N>
__global__ __launch_bounds__(L2D_BS) void k3_ycols_fwd(int ncells, const cx<double>* __restrict__ tw,
                                                       const cx<double>* __restrict__ B,
                                                       cx<double>* __restrict__ A) {
  __shared__ cx<double> b0[COLS * N], b1[COLS * N];
  const int64_t g = blockIdx.x;                  // (cell, x, kz group)
  const int64_t slab = g / (N / COLS);           // cell * N + x
  const int k0 = (int)(g % (N / COLS)) * COLS;
  if (slab >= (int64_t)ncells * N) return;
  const cx<double>* Bs = B + slab * N * N;
  cx<double>* As = A + slab * N * N;
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int y = i / COLS, c = i % COLS;        // consecutive kz: 128-byte segments
    b0[c * N + y] = Bs[(int64_t)y * N + k0 + c];
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, -1, COLS>(b0, b1, tw);
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int c = i / N, ky = i % N;             // rows kz0 + c, contiguous in ky
    As[(int64_t)(k0 + c) * N + ky] = r[i];
  }
}

// groups of 8 k1 per (cell, k2): DFT along x of in[x][k2][k1] -> out; MUL
// multiplies by the term table Gt[k0][k2][k1] first
template <int N, int SIGN, bool MUL>
__global__ __launch_bounds__(L2D_BS) void k3_xcols(int ncells, const cx<double>* __restrict__ tw,
                                                   const cx<double>* __restrict__ Gt,
                                                   const cx<double>* in, cx<double>* out) {
  __shared__ cx<double> b0[COLS * N], b1[COLS * N];
  const int64_t g = blockIdx.x;                  // (cell, k2, k1 group)
  const int64_t cc = g / ((int64_t)N * (N / COLS));
  const int k2 = (int)((g / (N / COLS)) % N);
  const int k10 = (int)(g % (N / COLS)) * COLS;
  if (cc >= ncells) return;
  const int64_t n = (int64_t)N * N * N;
  const cx<double>* ic = in + cc * n;
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int x = i / COLS, c = i % COLS;
    const int64_t e = ((int64_t)x * N + k2) * N + k10 + c;
    cx<double> v = ic[e];
    if constexpr (MUL) v = cmul(Gt[e], v);
    b0[c * N + x] = v;
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, SIGN, COLS>(b0, b1, tw);
  cx<double>* oc = out + cc * n;
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int x = i / COLS, c = i % COLS;
    oc[((int64_t)x * N + k2) * N + k10 + c] = r[c * N + x];
  }
}

// per x slab and group of 8 k1: inverse DFT along z of C[x][k2][k1], in place
template <int N>
__global__ __launch_bounds__(L2D_BS) void k3_zcols_inv(int ncells, const cx<double>* __restrict__ tw,
                                                       cx<double>* __restrict__ C) {
  __shared__ cx<double> b0[COLS * N], b1[COLS * N];
  const int64_t g = blockIdx.x;                  // (cell, x, k1 group)
  const int64_t slab = g / (N / COLS);
  const int k10 = (int)(g % (N / COLS)) * COLS;
  if (slab >= (int64_t)ncells * N) return;
  cx<double>* Cs = C + slab * N * N;
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int kz = i / COLS, c = i % COLS;
    b0[c * N + kz] = Cs[(int64_t)kz * N + k10 + c];
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, +1, COLS>(b0, b1, tw);
  for (int i = threadIdx.x; i < COLS * N; i += L2D_BS) {
    const int z = i / COLS, c = i % COLS;
    Cs[(int64_t)z * N + k10 + c] = r[c * N + z];
  }
}

// rows (cell, x, z): inverse DFT along y of C[x][z][k1]; LOSS: ACC = -F Re c,
// else ACC += Re c Im c
template <int N, bool LOSS>
__global__ __launch_bounds__(L2D_BS) void k3_rows_acc(int ncells, const cx<double>* __restrict__ tw,
                                                      const cx<double>* __restrict__ C,
                                                      const double* __restrict__ f,
                                                      const int64_t* __restrict__ off,
                                                      int64_t cell0, double* __restrict__ acc) {
  constexpr int NL = rows3_per_block<N>();
  __shared__ cx<double> b0[NL * N], b1[NL * N];
  const int64_t row0 = (int64_t)blockIdx.x * NL;
  const int64_t rows = (int64_t)ncells * N * N;
  for (int i = threadIdx.x; i < NL * N; i += L2D_BS) {
    const int64_t row = row0 + i / N;
    b0[i] = row < rows ? C[row * N + i % N] : cx<double>{0.0, 0.0};
  }
  __syncthreads();
  const cx<double>* r = lds_fft<N, +1, NL>(b0, b1, tw);
  for (int i = threadIdx.x; i < NL * N; i += L2D_BS) {
    const int64_t row = row0 + i / N;           // (cell, x, z)
    if (row >= rows) continue;
    const int y = i % N;
    const cx<double> c = r[i];
    if constexpr (LOSS) {
      const int64_t cc = row / (N * N), x = (row / N) % N, z = row % N;
      acc[row * N + y] = -f[off[cell0 + cc] + (x * N + y) * N + z] * c.x;
    } else {
      acc[row * N + y] += c.x * c.y;
    }
  }
}

// Q[x][y][z] = ACC[x][z][y] (dt == 0) or F + dt ACC, by 32 x 32 tiles
template <int N>
__global__ __launch_bounds__(L2D_BS) void k3_final(int ncells, const double* __restrict__ acc,
                                                   const double* f, const int64_t* __restrict__ off,
                                                   int64_t cell0, double* Q, double dt) {
  constexpr int TL = 32, TPS = (N / TL) * (N / TL);
  __shared__ double tile[TL][TL + 1];
  const int64_t g = blockIdx.x;                  // (cell, x, tile)
  const int64_t slab = g / TPS;
  const int t = (int)(g % TPS);
  const int z0 = (t / (N / TL)) * TL, y0 = (t % (N / TL)) * TL;
  if (slab >= (int64_t)ncells * N) return;
  const int64_t cc = slab / N, x = slab % N;
  const double* as = acc + slab * N * N;         // [z][y]
  for (int i = threadIdx.x; i < TL * TL; i += L2D_BS) {
    const int zz = i / TL, yy = i % TL;
    tile[zz][yy] = as[(int64_t)(z0 + zz) * N + y0 + yy];
  }
  __syncthreads();
  const int64_t base = off[cell0 + cc] + x * N * N;
  for (int i = threadIdx.x; i < TL * TL; i += L2D_BS) {
    const int yy = i / TL, zz = i % TL;
    const int64_t idx = base + (int64_t)(y0 + yy) * N + z0 + zz;
    const double q = tile[zz][yy];
    Q[idx] = dt == 0.0 ? q : f[idx] + dt * q;
  }
}

template <int N>
static hipError_t launch_t(const ChunkArgs& a, const cx<double>* tw, hipStream_t st) {
  constexpr int NL = rows3_per_block<N>();
  const int64_t n = (int64_t)N * N * N;
  cx<double>* A = (cx<double>*)a.W;
  cx<double>* C = (cx<double>*)a.Z;
  double* acc = (double*)(C + (int64_t)a.ncells * n);
  const cx<double>* G = (const cx<double>*)a.gamma;
  const int64_t rows = (int64_t)a.ncells * N * N;
  const dim3 rgrid((unsigned)((rows + NL - 1) / NL)), block(L2D_BS);
  const dim3 cgrid((unsigned)((int64_t)a.ncells * N * (N / COLS)));
  if (a.ev) (void)hipEventRecord(a.ev[0], st);
  hipLaunchKernelGGL((k3_rows_fwd<N>), rgrid, block, 0, st, a.f, a.off, a.cell0, a.ncells, tw, C);
  hipLaunchKernelGGL((k3_ycols_fwd<N>), cgrid, block, 0, st, a.ncells, tw, (const cx<double>*)C, A);
  hipLaunchKernelGGL((k3_xcols<N, -1, false>), cgrid, block, 0, st, a.ncells, tw,
                     (const cx<double>*)nullptr, (const cx<double>*)A, A);
  if (a.ev) (void)hipEventRecord(a.ev[1], st);
  for (int it = 0; it < a.J; ++it) {
    const int t = it == 0 ? a.J - 1 : it - 1;   // the loss term first
    hipLaunchKernelGGL((k3_xcols<N, +1, true>), cgrid, block, 0, st, a.ncells, tw,
                       G + (int64_t)t * n, (const cx<double>*)A, C);
    hipLaunchKernelGGL((k3_zcols_inv<N>), cgrid, block, 0, st, a.ncells, tw, C);
    if (it == 0)
      hipLaunchKernelGGL((k3_rows_acc<N, true>), rgrid, block, 0, st, a.ncells, tw,
                         (const cx<double>*)C, a.f, a.off, a.cell0, acc);
    else
      hipLaunchKernelGGL((k3_rows_acc<N, false>), rgrid, block, 0, st, a.ncells, tw,
                         (const cx<double>*)C, a.f, a.off, a.cell0, acc);
  }
  if (a.ev) (void)hipEventRecord(a.ev[2], st);
  hipLaunchKernelGGL((k3_final<N>), dim3((unsigned)((int64_t)a.ncells * N * (N / 32) * (N / 32))),
                     block, 0, st, a.ncells, (const double*)acc, a.f, a.off, a.cell0, a.Q, a.dt);
  if (a.ev) (void)hipEventRecord(a.ev[3], st);
  return hipGetLastError();
}

bool large3d_supported(int N) { return N == 64 || N == 128; }

hipError_t launch_large3d(const ChunkArgs& a, const void* twiddles, hipStream_t st) {
  if (a.ncells <= 0) return hipSuccess;
  if (a.d != 3 || a.precision != 0 || !twiddles) return hipErrorInvalidValue;
  const cx<double>* tw = (const cx<double>*)twiddles;
  switch (a.N) {
    case 64: return launch_t<64>(a, tw, st);
    case 128: return launch_t<128>(a, tw, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace efm

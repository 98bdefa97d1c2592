// Software-pipelined 3D collision kernel: one launch per chunk of cells runs
// four roles on four different chunks, so the per-term intermediate spectra of
// a chunk stay resident in the last-level cache (MALL) between the launch
// that writes them and the next one that reads them, and the memory-bound
// pencil role overlaps the arithmetic-heavy slab role.
//
// Launch i (chunks are consecutive runs of `chunk` cells of one plan):
//   F  chunk i     forward DFT along y and z of every x slab      -> W[i%2]
//   P  chunk i-1   forward DFT along x of every (k1,k2) pencil, then for each
//                  term j of the block's term group: multiply by
//                  gamma_j = alpha_j + i beta_j, inverse DFT along x -> Z[(i-1)%2]
//   S  chunk i-2   per x slab and term group: inverse DFT along z and y of
//                  every term, FP64 sum of Re c_j Im c_j (the gain products of
//                  the group) -> Pg[(i-2)%2][g]; the group holding the last
//                  term (the diagonal D) stores l = Re c_{J-1} -> Lr[(i-2)%2]
//   C  chunk i-3   Q = sum_g Pg - F l (fixed order), or F + dt Q in place
// A ring of two slots per buffer is enough: a slot written in launch i is
// read in launch i+1 and rewritten in launch i+2.
#include <hip/hip_runtime.h>

#include "fft.h"
#include "pipe.h"

namespace efm {

template <int N>
constexpr int pipe_bs() { return N == 24 || N == 12 ? 96 : 64; }
template <int N>
constexpr int pipe_spb() { return pipe_bs<N>() / N; }   // slabs per block (F, S)
constexpr int PIPE_CPB = 4;                            // cells per block (P)
template <int N>
constexpr int pipe_ppb() { return pipe_bs<N>() / PIPE_CPB; }   // pencils per block (P)
constexpr int PIPE_PPT = 8;                            // points per thread (C)

template <typename R, int N>
struct PipeSmem {
  static constexpr int SPB = pipe_spb<N>();
  static constexpr size_t slab_bytes = sizeof(cx<R>) * SPB * N * (N + 1);
  static constexpr size_t pen_bytes = sizeof(cx<R>) * N * pipe_bs<N>();
  static constexpr size_t bytes = slab_bytes > pen_bytes ? slab_bytes : pen_bytes;
};

// ---- role F ----------------------------------------------------------------
template <typename R, int N>
__device__ __forceinline__ void role_fwd(const PipeArgs& a, int blk, cx<R>* smem) {
  constexpr int SPB = pipe_spb<N>();
  constexpr int P = N * N;
  cx<R>(*lds)[N][N + 1] = reinterpret_cast<cx<R>(*)[N][N + 1]>(smem);
  const int s = threadIdx.x / N, i = threadIdx.x % N;
  const int64_t slab = (int64_t)blk * SPB + s;
  const bool active = s < SPB && slab < (int64_t)a.f_n * N;
  const int cc = active ? (int)(slab / N) : 0;
  const int x = active ? (int)(slab % N) : 0;
  const int ss = s < SPB ? s : 0;
  cx<R> v[N];
  {
    const double* fc = a.f + a.off[a.f_cell0 + cc] + (int64_t)x * P;
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = {(R)fc[y * N + i], (R)0};
  }
  fft_line<N, -1>(v);
  if (s < SPB) {
#pragma unroll
    for (int k1 = 0; k1 < N; ++k1) lds[ss][k1][i] = v[k1];
  }
  __syncthreads();
#pragma unroll
  for (int z = 0; z < N; ++z) v[z] = lds[ss][i][z];
  fft_line<N, -1>(v);
  if (active) {
    cx<R>* Wc = (cx<R>*)a.W[a.f_slot] + ((int64_t)cc * N + x) * P;
#pragma unroll
    for (int k2 = 0; k2 < N; ++k2) Wc[k2 * N + i] = v[k2];
  }
}

// ---- role P ----------------------------------------------------------------
template <typename R, int N>
__device__ __forceinline__ void role_pencil(const PipeArgs& a, int blk, cx<R>* smem) {
  constexpr int P = N * N;
  constexpr int PPB = pipe_ppb<N>();
  constexpr int BS = pipe_bs<N>();
  constexpr int PB = (P + PPB - 1) / PPB;          // pencil blocks per cell group
  cx<R>(*fh)[BS] = reinterpret_cast<cx<R>(*)[BS]>(smem);
  const int g = blk % a.G;
  const int rest = blk / a.G;
  const int pb = rest % PB;
  const int cg = rest / PB;
  const int t = threadIdx.x;
  const int c_in = t / PPB, pl = t % PPB;
  const int p = pb * PPB + pl;
  const int cc = cg * PIPE_CPB + c_in;
  const bool active = p < P && cc < a.p_n;
  const int pp = p < P ? p : 0;
  const int ccs = active ? cc : 0;
  const int j0 = g * a.J / a.G, j1 = (g + 1) * a.J / a.G;
  cx<R> v[N];
  {
    const cx<R>* Wc = (const cx<R>*)a.W[a.p_slot] + (int64_t)ccs * N * P + pp;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = Wc[(int64_t)k * P];
  }
  fft_line<N, -1>(v);                               // Fh(k0, p), unnormalised
#pragma unroll
  for (int k = 0; k < N; ++k) fh[k][t] = v[k];      // own column only
  const cx<R>* G = (const cx<R>*)a.gamma;
  cx<R>* Z = (cx<R>*)a.Z[a.p_slot];
  for (int j = j0; j < j1; ++j) {
    const cx<R>* Gj = G + (int64_t)j * N * P + pp;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = cmul(Gj[(int64_t)k * P], fh[k][t]);
    fft_line<N, +1>(v);
    if (active) {
      cx<R>* Zj = Z + ((int64_t)ccs * a.J + j) * N * P + pp;
#pragma unroll
      for (int xx = 0; xx < N; ++xx) Zj[(int64_t)xx * P] = v[xx];
    }
  }
}

// ---- role S ----------------------------------------------------------------
template <typename R, int N>
__device__ __forceinline__ void role_slab(const PipeArgs& a, int blk, cx<R>* smem) {
  constexpr int SPB = pipe_spb<N>();
  constexpr int P = N * N;
  cx<R>(*lds)[N][N + 1] = reinterpret_cast<cx<R>(*)[N][N + 1]>(smem);
  const int g = blk % a.G;
  const int sb = blk / a.G;
  const int s = threadIdx.x / N, i = threadIdx.x % N;
  const int64_t slab = (int64_t)sb * SPB + s;
  const bool active = s < SPB && slab < (int64_t)a.s_n * N;
  const int cc = active ? (int)(slab / N) : 0;
  const int x = active ? (int)(slab % N) : 0;
  const int ss = s < SPB ? s : 0;
  const int j0 = g * a.J / a.G, j1 = (g + 1) * a.J / a.G;
  double acc[N];
#pragma unroll
  for (int y = 0; y < N; ++y) acc[y] = 0.0;
  cx<R> v[N];
  const cx<R>* Z = (const cx<R>*)a.Z[a.s_slot];
  for (int j = j0; j < j1; ++j) {
    const cx<R>* Zs = Z + (((int64_t)cc * a.J + j) * N + x) * P;
#pragma unroll
    for (int k2 = 0; k2 < N; ++k2) v[k2] = Zs[k2 * N + i];
    fft_line<N, +1>(v);
    __syncthreads();
    if (s < SPB) {
#pragma unroll
      for (int z = 0; z < N; ++z) lds[ss][i][z] = v[z];
    }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < N; ++k1) v[k1] = lds[ss][k1][i];
    fft_line<N, +1>(v);
    if (j + 1 < a.J) {
#pragma unroll
      for (int y = 0; y < N; ++y) acc[y] += (double)v[y].x * (double)v[y].y;
    }
  }
  if (active) {
    const int64_t base = (int64_t)cc * N * P + (int64_t)x * P;
    double* pg = a.Pg[a.s_slot] + (int64_t)g * a.chunk * N * P + base;
#pragma unroll
    for (int y = 0; y < N; ++y) pg[y * N + i] = acc[y];
    if (j1 == a.J) {
      double* lr = a.Lr[a.s_slot] + base;
#pragma unroll
      for (int y = 0; y < N; ++y) lr[y * N + i] = (double)v[y].x;
    }
  }
}

// ---- role C ----------------------------------------------------------------
template <int N>
__device__ __forceinline__ void role_combine(const PipeArgs& a, int blk) {
  constexpr int64_t n = (int64_t)N * N * N;
  constexpr int BS = pipe_bs<N>();
  const double* pg0 = a.Pg[a.c_slot];
  const double* lr = a.Lr[a.c_slot];
  const int64_t stride_g = (int64_t)a.chunk * n;
#pragma unroll
  for (int k = 0; k < PIPE_PPT; ++k) {
    const int64_t e = ((int64_t)blk * PIPE_PPT + k) * BS + threadIdx.x;
    if (e < (int64_t)a.c_n * n) {
      const int cc = (int)(e / n);
      const int64_t r = e - (int64_t)cc * n;
      double gsum = 0.0;
      for (int g = 0; g < a.G; ++g) gsum += pg0[g * stride_g + e];
      const int64_t fo = a.off[a.c_cell0 + cc] + r;
      const double fv = a.f[fo];
      const double q = gsum - fv * lr[e];
      a.Q[fo] = (a.dt == 0.0) ? q : fv + a.dt * q;
    }
  }
}

template <typename R, int N>
__global__ __launch_bounds__(pipe_bs<N>()) void k_pipe(const PipeArgs a) {
  __shared__ __align__(16) char smem_raw[PipeSmem<R, N>::bytes];
  cx<R>* smem = reinterpret_cast<cx<R>*>(smem_raw);
  int b = blockIdx.x;
  if (b < a.f_blocks) { role_fwd<R, N>(a, b, smem); return; }
  b -= a.f_blocks;
  if (b < a.p_blocks) { role_pencil<R, N>(a, b, smem); return; }
  b -= a.p_blocks;
  if (b < a.s_blocks) { role_slab<R, N>(a, b, smem); return; }
  b -= a.s_blocks;
  if (b < a.c_blocks) { role_combine<N>(a, b); return; }
}

// ---- host side -------------------------------------------------------------
template <int N>
static void role_blocks(PipeArgs& a) {
  constexpr int SPB = pipe_spb<N>();
  constexpr int PPB = pipe_ppb<N>();
  constexpr int P = N * N;
  constexpr int PB = (P + PPB - 1) / PPB;
  constexpr int64_t n = (int64_t)N * N * N;
  a.f_blocks = a.f_n > 0 ? (int)(((int64_t)a.f_n * N + SPB - 1) / SPB) : 0;
  a.p_blocks = a.p_n > 0 ? ((a.p_n + PIPE_CPB - 1) / PIPE_CPB) * PB * a.G : 0;
  a.s_blocks = a.s_n > 0 ? (int)(((int64_t)a.s_n * N + SPB - 1) / SPB) * a.G : 0;
  a.c_blocks = a.c_n > 0 ? (int)(((int64_t)a.c_n * n + (int64_t)PIPE_PPT * pipe_bs<N>() - 1) /
                                 ((int64_t)PIPE_PPT * pipe_bs<N>()))
                         : 0;
}

template <typename R, int N>
static hipError_t launch_pipe_t(PipeArgs& a, hipStream_t st) {
  role_blocks<N>(a);
  const int total = a.f_blocks + a.p_blocks + a.s_blocks + a.c_blocks;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL((k_pipe<R, N>), dim3(total), dim3(pipe_bs<N>()), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pipe(PipeArgs& a, int N, int precision, hipStream_t st) {
#define EFM_PCASE(NN)                                                                    \
  case NN:                                                                               \
    return precision == 1 ? launch_pipe_t<float, NN>(a, st) : launch_pipe_t<double, NN>(a, st);
  switch (N) {
    EFM_PCASE(8)
    EFM_PCASE(12)
    EFM_PCASE(16)
    EFM_PCASE(24)
    EFM_PCASE(32)
    default:
      return hipErrorInvalidValue;
  }
#undef EFM_PCASE
}

}  // namespace efm

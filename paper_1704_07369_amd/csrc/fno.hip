// Kernels of the learned surrogate: a Fourier neural operator (FNO) on the
// velocity grid, FP32, forward and backward, written for gfx950.
//
// Network (per cell, n = N^3 points, C channels, modes kx, ky in [-K, K),
// kz in [0, K) -- NM = 4 K^3 modes):
//   u0 = lift(F~)             u0[c] = Wl[c] F~ + bl[c]      (F~ = c0 F / mass)
//   for l < L:  h = W_l u + b_l + S_l(u);  u <- GELU(h)  (no GELU after the last layer)
//   y  = proj(u)              y = sum_c Wp[c] u[c] + bp      (prediction of c0^2 Q / mass^2)
// with c0 = (2 pi)^{3/2}, which puts a unit-temperature Maxwellian's peak at 1
// (Q is quadratic in F, so the target scales with the square of the input).
// Spectral convolution S(u)[o] = Re IDFT( scatter_m( sum_i R[m][i][o] Uh[m][i] ) ) / n,
// Uh[m][i] = DFT(u[i]) at the kept modes: unnormalised kernels, with the 1/n of
// the normalised inverse applied in the mode mixing, so R is O(1/C) like the
// dense weights (Adam's steps are of one size for all parameters; an R that
// carries the 1/n itself makes every step 1/n too coarse).  Its adjoint in u is
// the same pair of transforms with conj(R) transposed and the same 1/n, and
// dR[m][i][o] = sum_b Gv[b][m][o] conj(Uh[b][m][i]) / n where Gv is the
// truncated DFT of the output gradient.  Every truncated transform is a
// pruned 3D FFT: forward = z lines of the slab (keep kz < K) -> y lines of the
// kept kz (keep 2K ky) -> x lines of the 2K x K kept (ky, kz) pencils (keep
// 2K kx); inverse = the same passes backwards with zero padding.  Inference at
// C = 16 keeps the slab passes' output channel-last and runs the x lines and
// the mode mixing as one kernel (k_fno_xmix16); training and the other channel
// counts keep it channel-first, with separate x passes and mixing, since the
// weight gradient needs the kept modes in device memory anyway.
#include <hip/hip_runtime.h>

#include "fft.h"
#include "fno.h"

namespace efm {

template <int N, int K>
struct FnoDims {
  static constexpr int n = N * N * N;
  static constexpr int KY = 2 * K;           // kept ky (and kx) values
  static constexpr int PEN = KY * K;         // kept (ky, kz) pencils per slab
  static constexpr int NM = KY * PEN;        // kept modes
  static_assert(2 * K <= N, "modes");
};

template <int N, int K>
__device__ __forceinline__ int kidx(int m) {   // index m in [0, 2K) -> FFT index
  return m < K ? m : N - 2 * K + m;
}

// Offset of the truncated spectrum T of (cell b, channel c, slab x, kept
// (ky, kz) pencil e): channel-first [b][c][x][pen] (training, whose x passes
// take a tile of pencils of one channel), or channel-last [b][x][pen][c]
// (inference at C = 16, whose spectral kernel takes one pencil of every
// channel of 16 cells)
template <int N, int K, int C, bool CL>
__device__ __forceinline__ int64_t tofs(int64_t b, int c, int x, int e) {
  constexpr int PEN = FnoDims<N, K>::PEN;
  return CL ? ((b * N + x) * PEN + e) * C + c : ((b * C + c) * N + x) * PEN + e;
}

// ---------------------------------------------------------------------------
// Transform passes.  Slab passes take SB = 256 / N slabs per 256-thread block
// (one thread per line, LDS transposes inside each slab); x passes take one
// cell and a tile of TP = 256 / C pencils of every channel, and move the kept
// modes Uh[b][mode][c] through LDS so that their global reads and writes are
// contiguous (channel fastest).
// ---------------------------------------------------------------------------
template <int N>
constexpr int slabs_per_block() { return 256 / N; }
template <int C>
constexpr int pens_per_block() { return 256 / C; }

// The lifted input u0[b][c] = Wl[c] F~[b] + bl[c], formed where it is read
// (inference never stores u0)
struct LiftIn {
  const float* Fin = nullptr;   // [B][n]; null: read the stored activation
  const float* Wl = nullptr;
  const float* bl = nullptr;
};

// truncated forward transform, slab pass: real u[s][x][y][z] -> T[s][x][ky][kz]
// (lift.Fin set: u = the lifted input, s = b*C + c)
template <int N, int K>
__global__ __launch_bounds__(256) void k_fno_fwd_slab(const float* __restrict__ u,
                                                      cx<float>* __restrict__ T, int64_t nslab,
                                                      LiftIn lift, int C) {
  using D = FnoDims<N, K>;
  constexpr int SB = slabs_per_block<N>();
  __shared__ cx<float> lds[SB][N][K + 1];
  const int ls = threadIdx.x / N, i = threadIdx.x % N;
  const int64_t slab0 = (int64_t)blockIdx.x * SB;
  if (slab0 + ls < nslab) {                       // thread (ls, i): line y = i of slab ls
    cx<float> v[N];
    if (lift.Fin) {
      const int64_t sc = (slab0 + ls) / N;        // s = b*C + c
      const int x = (int)((slab0 + ls) % N);
      const float* fs = lift.Fin + (sc / C) * D::n + (int64_t)x * N * N;
      const float w = lift.Wl[sc % C], c0 = lift.bl[sc % C];
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = {w * fs[i * N + z] + c0, 0.f};
    } else {
      const float* us = u + (slab0 + ls) * N * N;
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = {us[i * N + z], 0.f};
    }
    fft_line<N, -1>(v);
#pragma unroll
    for (int kz = 0; kz < K; ++kz) lds[ls][i][kz] = v[kz];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SB * K; t += 256) {   // (slab, kz column) items
    const int l2 = t / K, col = t % K;
    if (slab0 + l2 >= nslab) continue;
    cx<float> v[N];
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = lds[l2][y][col];
    fft_line<N, -1>(v);
    cx<float>* Ts = T + (slab0 + l2) * D::PEN;
#pragma unroll
    for (int m = 0; m < D::KY; ++m) Ts[m * K + col] = v[kidx<N, K>(m)];
  }
}

// truncated forward transform, x pass: T[s][x][pen] -> Uh[b][mode][c] (s = b*C + c);
// grid (pencil tiles, cells)
template <int N, int K, int C>
__global__ __launch_bounds__(256) void k_fno_fwd_x(const cx<float>* __restrict__ T,
                                                   cx<float>* __restrict__ Uh) {
  using D = FnoDims<N, K>;
  constexpr int TP = pens_per_block<C>(), LC = C + 1;
  __shared__ cx<float> buf[D::KY][TP * LC];
  const int b = blockIdx.y;
  const int pen0 = blockIdx.x * TP;
  const int np = min(TP, D::PEN - pen0);
  const int c = threadIdx.x / TP, p = threadIdx.x % TP;
  if (p < np) {
    const cx<float>* Ts = T + ((int64_t)b * C + c) * N * D::PEN + pen0 + p;
    cx<float> v[N];
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = Ts[(int64_t)x * D::PEN];
    fft_line<N, -1>(v);
#pragma unroll
    for (int mx = 0; mx < D::KY; ++mx) buf[mx][p * LC + c] = v[kidx<N, K>(mx)];
  }
  __syncthreads();
  for (int mx = 0; mx < D::KY; ++mx) {
    cx<float>* out = Uh + ((int64_t)b * D::NM + mx * D::PEN + pen0) * C;
    for (int e = threadIdx.x; e < np * C; e += 256) out[e] = buf[mx][(e / C) * LC + e % C];
  }
}

// truncated inverse transform, x pass: V[b][mode][c] -> T[s][x][pen]; grid (pencil tiles, cells)
template <int N, int K, int C>
__global__ __launch_bounds__(256) void k_fno_inv_x(const cx<float>* __restrict__ V,
                                                   cx<float>* __restrict__ T) {
  using D = FnoDims<N, K>;
  constexpr int TP = pens_per_block<C>(), LC = C + 1;
  __shared__ cx<float> buf[D::KY][TP * LC];
  const int b = blockIdx.y;
  const int pen0 = blockIdx.x * TP;
  const int np = min(TP, D::PEN - pen0);
  for (int mx = 0; mx < D::KY; ++mx) {
    const cx<float>* in = V + ((int64_t)b * D::NM + mx * D::PEN + pen0) * C;
    for (int e = threadIdx.x; e < np * C; e += 256) buf[mx][(e / C) * LC + e % C] = in[e];
  }
  __syncthreads();
  const int c = threadIdx.x / TP, p = threadIdx.x % TP;
  if (p >= np) return;
  cx<float> v[N];
#pragma unroll
  for (int x = 0; x < N; ++x) v[x] = {0.f, 0.f};
#pragma unroll
  for (int mx = 0; mx < D::KY; ++mx) v[kidx<N, K>(mx)] = buf[mx][p * LC + c];
  fft_line<N, +1>(v);
  cx<float>* Ts = T + ((int64_t)b * C + c) * N * D::PEN + pen0 + p;
#pragma unroll
  for (int x = 0; x < N; ++x) Ts[(int64_t)x * D::PEN] = v[x];
}

// The spectral branch between the slab passes of inference at C = 16, fused,
// on the channel-last T: one block per (kept (ky, kz) pencil, chunk of 16
// cells), 256 threads.
//  1. thread (cell r, channel c) transforms its x line forward (the 16
//     channels of a cell are 128 contiguous bytes at each x) and keeps the
//     kx of the kept modes, into LDS;
//  2. wave w mixes the pencil's modes kx = w, w + 4, ... on the matrix cores:
//     per mode Y = scale X W over the 16 cells as in k_fno_mix_mfma16 (the
//     real product [Xr Xi] [[Wr, Wi], [-Wi, Wr]], 16 v_mfma_f32_16x16x4_f32;
//     lane (r, q) takes channels 4 q .. 4 q + 3 of cell r from LDS and the
//     weights W(4 q + k, r) = R[m][4 q + k][r], and ends with output channel
//     r of cells 4 q .. 4 q + 3, which it writes over the mode's inputs);
//  3. thread (cell, c) transforms the mixed line back and stores it in place.
// The kept modes never go through global memory, and each weight is read once
// per 16 cells.  Cells beyond B transform zeros and store nothing.
template <int N, int K>
__global__ __launch_bounds__(256) void k_fno_xmix16(cx<float>* T, int B,
                                                    const cx<float>* __restrict__ R, float scale) {
  using D = FnoDims<N, K>;
  constexpr int C = 16, CB = 16, LC = C + 1;
  typedef float v4f __attribute__((ext_vector_type(4)));
  __shared__ cx<float> X[D::KY][CB][LC];
  const int pen = blockIdx.x;
  const int b0 = blockIdx.y * CB;
  const int c = threadIdx.x % C, cl = threadIdx.x / C;
  const bool live = b0 + cl < B;
  cx<float>* Tl = T + tofs<N, K, C, true>(live ? b0 + cl : b0, c, 0, pen);   // + x PEN C
  constexpr int64_t XS = (int64_t)D::PEN * C;
  {
    cx<float> v[N];
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = live ? Tl[x * XS] : cx<float>{0.f, 0.f};
    fft_line<N, -1>(v);
#pragma unroll
    for (int mx = 0; mx < D::KY; ++mx) X[mx][cl][c] = v[kidx<N, K>(mx)];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  // this lane's weights of the wave's next mode are in flight during the current one
  const cx<float>* Rl = R + (int64_t)pen * C * C + 4 * q * C + r;
  constexpr int64_t KXS = (int64_t)D::PEN * C * C;   // kx -> kx + 1
  cx<float> wn[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) wn[k] = Rl[wv * KXS + k * C];
  for (int mx = wv; mx < D::KY; mx += 4) {   // uniform per wave
    cx<float> w[4], xv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      w[k] = wn[k];
      xv[k] = X[mx][r][4 * q + k];
    }
    if (mx + 4 < D::KY) {
#pragma unroll
      for (int k = 0; k < 4; ++k) wn[k] = Rl[(mx + 4) * KXS + k * C];
    }
    v4f acc[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      acc[hh] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        // A = [Xr Xi]; B rows k < 4: [Wr | Wi], rows k >= 4: [-Wi | Wr]
        const float a = k < 4 ? xv[k].x : xv[k - 4].y;
        const cx<float> wk = w[k & 3];
        const float bv = k < 4 ? (hh == 0 ? wk.x : wk.y) : (hh == 0 ? -wk.y : wk.x);
        acc[hh] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[hh], 0, 0, 0);
      }
    }
    // this wave's reads of X[mx] precede its writes (one wave, in order)
#pragma unroll
    for (int v = 0; v < 4; ++v) X[mx][4 * q + v][r] = {scale * acc[0][v], scale * acc[1][v]};
  }
  __syncthreads();
  {
    cx<float> v[N];
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = {0.f, 0.f};
#pragma unroll
    for (int mx = 0; mx < D::KY; ++mx) v[kidx<N, K>(mx)] = X[mx][cl][c];
    fft_line<N, +1>(v);
    if (live) {
#pragma unroll
      for (int x = 0; x < N; ++x) Tl[x * XS] = v[x];
    }
  }
}

// truncated inverse transform, slab pass: T[s][x][ky][kz] -> out[s][x][y][z] = Re(...)
// (accumulate != 0: out += result); the real slabs are staged in LDS so that
// the global stores are contiguous
template <int N, int K>
__global__ __launch_bounds__(256) void k_fno_inv_slab(const cx<float>* __restrict__ T,
                                                      float* __restrict__ out, int64_t nslab,
                                                      int accumulate) {
  using D = FnoDims<N, K>;
  constexpr int SB = slabs_per_block<N>(), LN = N + 1;
  constexpr int CBYTES = (int)sizeof(cx<float>) * SB * N * (K + 1);
  constexpr int RBYTES = (int)sizeof(float) * SB * N * LN;
  __shared__ __align__(16) unsigned char raw[CBYTES > RBYTES ? CBYTES : RBYTES];
  auto lds = reinterpret_cast<cx<float>(*)[N][K + 1]>(raw);   // [SB][N][K + 1] spectrum
  auto rl = reinterpret_cast<float(*)[N][LN]>(raw);            // [SB][N][N + 1] real slabs
  const int64_t slab0 = (int64_t)blockIdx.x * SB;
  for (int t = threadIdx.x; t < SB * K; t += 256) {   // (slab, kz column) items
    const int l2 = t / K, col = t % K;
    if (slab0 + l2 >= nslab) continue;
    const cx<float>* Ts = T + (slab0 + l2) * D::PEN;
    cx<float> v[N];
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = {0.f, 0.f};
#pragma unroll
    for (int m = 0; m < D::KY; ++m) v[kidx<N, K>(m)] = Ts[m * K + col];
    fft_line<N, +1>(v);
#pragma unroll
    for (int y = 0; y < N; ++y) lds[l2][y][col] = v[y];
  }
  __syncthreads();
  const int ls = threadIdx.x / N, i = threadIdx.x % N;   // thread (ls, i): line y = i
  cx<float> v[N];
#pragma unroll
  for (int z = 0; z < N; ++z) v[z] = {0.f, 0.f};
  if (slab0 + ls < nslab) {
#pragma unroll
    for (int kz = 0; kz < K; ++kz) v[kz] = lds[ls][i][kz];
    fft_line<N, +1>(v);
  }
  __syncthreads();                                // every read of the spectrum is done
#pragma unroll
  for (int z = 0; z < N; ++z) rl[ls][i][z] = v[z].x;
  __syncthreads();
  const int64_t nval = (slab0 + SB <= nslab ? SB : nslab - slab0) * N * N;
  float* os = out + slab0 * N * N;
  for (int64_t e = threadIdx.x; e < nval; e += 256) {
    const int sl = (int)(e / (N * N)), y = (int)((e / N) % N), z = (int)(e % N);
    if (accumulate) os[e] += rl[sl][y][z];
    else os[e] = rl[sl][y][z];
  }
}

// ---------------------------------------------------------------------------
// mode mixing.  forward: Y[b][m][o] = scale sum_i R[m][i][o] X[b][m][i]
// adjoint:              Y[b][m][i] = scale sum_o conj(R[m][i][o]) X[b][m][o]
// one thread per (cell chunk, m, output channel): its C weights are read once
// and reused for the MIX_CELLS cells of the chunk
// ---------------------------------------------------------------------------
constexpr int MIX_CELLS = 32;

template <int C>
__global__ __launch_bounds__(256) void k_fno_mix2(const cx<float>* __restrict__ R,
                                                  const cx<float>* __restrict__ X, int B, int NM,
                                                  int adjoint, float scale,
                                                  cx<float>* __restrict__ Y) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nmc = (int64_t)NM * C;
  const int nchunk = (B + MIX_CELLS - 1) / MIX_CELLS;
  if (gid >= nmc * nchunk) return;
  const int o = (int)(gid % C);
  const int m = (int)((gid / C) % NM);
  const int b0 = (int)(gid / nmc) * MIX_CELLS;
  const cx<float>* Rm = R + (int64_t)m * C * C;
  cx<float> r[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    // forward: R[m][k][o] (k = input channel); adjoint: conj R[m][o][k] (k = output channel)
    const cx<float> w = adjoint ? Rm[o * C + k] : Rm[k * C + o];
    r[k] = {w.x, adjoint ? -w.y : w.y};
  }
  const int b1 = min(B, b0 + MIX_CELLS);
#pragma unroll 4
  for (int b = b0; b < b1; ++b) {
    const cx<float>* x = X + ((int64_t)b * NM + m) * C;
    cx<float> acc = {0.f, 0.f};
#pragma unroll
    for (int k = 0; k < C; ++k) acc = cadd(acc, cmul(r[k], x[k]));
    Y[((int64_t)b * NM + m) * C + o] = {scale * acc.x, scale * acc.y};
  }
}

// The same mixing on the matrix cores (C = 16).  Per mode m and chunk of 64
// cells, Y = scale X W with X, Y 64 x 16 complex and W 16 x 16 complex
// (forward W(c, j) = R[m][c][j], adjoint W(c, j) = conj R[m][j][c]), as the
// real product [Xr Xi] [[Wr, Wi], [-Wi, Wr]] = [Yr Yi] of K = 32: four cell
// tiles x two output halves x eight K steps of v_mfma_f32_16x16x4_f32, FP32
// products and sums as on the vector ALU.  Operand layout of 16x16x4 (lane l,
// r = l % 16, q = l / 16): A[r][q], B[q][r], D[4 q + v][r] (v < 4).  One wave
// per (mode, cell chunk).  K step k (< 4: real parts, then imaginary parts)
// takes channel 4 q + k % 4 in the slot of lane group q, so lane (r, q) loads
// the four contiguous channels 4 q .. 4 q + 3 of X[b0 + 16 t + r][m] (32
// bytes, t < 4; cells beyond B read as zero and store nothing) and
// W(4 q + k, r), k < 4.
constexpr int MIX_MFMA_CELLS = 64;

__global__ __launch_bounds__(256) void k_fno_mix_mfma16(const cx<float>* __restrict__ R,
                                                        const cx<float>* __restrict__ X, int B,
                                                        int NM, int adjoint, float scale,
                                                        cx<float>* __restrict__ Y) {
  constexpr int C = 16, CT = MIX_MFMA_CELLS / 16;
  typedef float v4f __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nchunk = (B + MIX_MFMA_CELLS - 1) / MIX_MFMA_CELLS;
  if (wid >= (int64_t)NM * nchunk) return;  // uniform per wave
  const int m = (int)(wid % NM);
  const int b0 = (int)(wid / NM) * MIX_MFMA_CELLS;
  const int r = lane & 15, q = lane >> 4;
  const cx<float>* Rm = R + (int64_t)m * C * C;
  cx<float> w[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int c = 4 * q + k;
    const cx<float> t = adjoint ? Rm[r * C + c] : Rm[c * C + r];
    w[k] = {t.x, adjoint ? -t.y : t.y};
  }
  cx<float> x[CT][4];
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int b = b0 + 16 * t + r;
    // two 16-byte loads: X is a device allocation of its own and a lane's
    // channels start at a multiple of 32 bytes
    const float4* xp = reinterpret_cast<const float4*>(X + ((int64_t)b * NM + m) * C + 4 * q);
    const float4 lo = b < B ? xp[0] : float4{0.f, 0.f, 0.f, 0.f};
    const float4 hi = b < B ? xp[1] : float4{0.f, 0.f, 0.f, 0.f};
    x[t][0] = {lo.x, lo.y};
    x[t][1] = {lo.z, lo.w};
    x[t][2] = {hi.x, hi.y};
    x[t][3] = {hi.z, hi.w};
  }
  v4f acc[CT][2];
#pragma unroll
  for (int t = 0; t < CT; ++t) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      acc[t][h] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        // A = [Xr Xi]; B rows k < 4: [Wr | Wi], rows k >= 4: [-Wi | Wr]
        const float a = k < 4 ? x[t][k].x : x[t][k - 4].y;
        const cx<float> wk = w[k & 3];
        const float bv = k < 4 ? (h == 0 ? wk.x : wk.y) : (h == 0 ? -wk.y : wk.x);
        acc[t][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[t][h], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = b0 + 16 * t + 4 * q + v;
      if (b < B) Y[((int64_t)b * NM + m) * C + r] = {scale * acc[t][0][v], scale * acc[t][1][v]};
    }
  }
}

// dR[m][i][o] = scale sum_b G[b][m][o] conj(U[b][m][i]); one thread per (m, o),
// summing every input channel i over the cells in order
template <int C>
__global__ __launch_bounds__(256) void k_fno_dR(const cx<float>* __restrict__ G,
                                                const cx<float>* __restrict__ U, int B, int NM,
                                                float scale, cx<float>* __restrict__ dR) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)NM * C) return;
  const int o = (int)(gid % C);
  const int64_t m = gid / C;
  cx<float> acc[C];
#pragma unroll
  for (int i = 0; i < C; ++i) acc[i] = {0.f, 0.f};
  for (int b = 0; b < B; ++b) {
    const cx<float> g = G[((int64_t)b * NM + m) * C + o];
    const cx<float>* ub = U + ((int64_t)b * NM + m) * C;
#pragma unroll
    for (int i = 0; i < C; ++i) acc[i] = cadd(acc[i], cmul(g, {ub[i].x, -ub[i].y}));
  }
#pragma unroll
  for (int i = 0; i < C; ++i) dR[(m * C + i) * C + o] = {scale * acc[i].x, scale * acc[i].y};
}

// ---------------------------------------------------------------------------
// pointwise parts
// ---------------------------------------------------------------------------
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  const float cdf = 0.5f * (1.f + erff(x * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
  return cdf + x * pdf;
}

// u0[b][c][r] = Wl[c] Fin[b][r] + bl[c]
template <int C>
__global__ __launch_bounds__(256) void k_fno_lift(const float* __restrict__ Fin, int B, int n,
                                                  const float* __restrict__ Wl,
                                                  const float* __restrict__ bl,
                                                  float* __restrict__ u0) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * n) return;
  const int64_t b = gid / n, r = gid % n;
  const float f = Fin[gid];
#pragma unroll
  for (int c = 0; c < C; ++c) u0[(b * C + c) * n + r] = Wl[c] * f + bl[c];
}

// The pointwise layer of one slab on the matrix cores (C = 16): per chunk of
// 64 points of the slab, pre = W in as four 16 x 16 x 16 products of four
// v_mfma_f32_16x16x4_f32 each (operand layout as in the mode mixing: lane l,
// r = l % 16, q = l / 16 supplies A[r][q] and B[q][r] and holds D[4 q + v][r]).
// K step j takes input channel 4 q + j in the slot of lane group q, and tile t
// holds the points c0 + 4 r + t in its columns, so lane (r, q) loads the four
// contiguous points c0 + 4 r .. c0 + 4 r + 3 of channels 4 q + j and ends
// with output channels 4 q + v of the same four points, stored the same way.
// Then h = pre + bias + s (s: the spectral branch in rl), uo = GELU(h) or h;
// the projection sum_c Wp[c] uo[c] + bp adds the four lane groups' partial
// sums across lanes.  keep: uo replaces s in rl for the next forward slab pass.
template <int N>
__device__ __forceinline__ void pointwise_mfma16(
    float (*rl)[N][N + 1], int x, int64_t b, const float* __restrict__ u, const LiftIn& lift,
    const float* __restrict__ W, const float* __restrict__ bias, int act, float* __restrict__ h,
    float* __restrict__ uo, const float* __restrict__ Wp, const float* __restrict__ bp,
    float* __restrict__ yout, bool keep) {
  constexpr int C = 16, n = N * N * N, NW = C * N / 64;
  static_assert(N % 8 == 0, "64-point chunks of whole 4-point row pieces");
  typedef float v4f __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  float wa[4], bo[4], wp[4], wl[4], bl[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    wa[j] = W[r * C + 4 * q + j];
    bo[j] = bias[4 * q + j];
    wp[j] = yout ? Wp[4 * q + j] : 0.f;
    wl[j] = lift.Fin ? lift.Wl[4 * q + j] : 0.f;
    bl[j] = lift.Fin ? lift.bl[4 * q + j] : 0.f;
  }
  const float bp0 = yout ? bp[0] : 0.f;
  for (int ch = wv; ch < N * N / 64; ch += NW) {   // uniform per wave
    const int p = ch * 64 + 4 * r;                 // the lane's first point in the slab
    const int yy = p / N, zz = p % N;              // its four points lie in row yy
    const int64_t rg = (int64_t)x * N * N + p;
    v4f in[4];
    if (lift.Fin) {   // a caller's array: no alignment beyond 4 bytes assumed
      const float* fp = lift.Fin + b * n + rg;
      const float f0 = fp[0], f1 = fp[1], f2 = fp[2], f3 = fp[3];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        in[j] = v4f{wl[j] * f0 + bl[j], wl[j] * f1 + bl[j], wl[j] * f2 + bl[j], wl[j] * f3 + bl[j]};
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        in[j] = *reinterpret_cast<const v4f*>(u + (b * C + 4 * q + j) * n + rg);
    }
    v4f acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[j], in[j][t], acc[t], 0, 0, 0);
    }
    v4f py = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int o = 4 * q + v;
      v4f hv, ov;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        hv[t] = acc[t][v] + bo[v] + rl[o][yy][zz + t];
        ov[t] = act ? gelu(hv[t]) : hv[t];
      }
      const int64_t go = (b * C + o) * n + rg;
      if (h) *reinterpret_cast<v4f*>(h + go) = hv;
      if (uo) *reinterpret_cast<v4f*>(uo + go) = ov;
      py += wp[v] * ov;
      if (keep) {
#pragma unroll
        for (int t = 0; t < 4; ++t) rl[o][yy][zz + t] = ov[t];   // this lane's own entries
      }
    }
    if (yout) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        py[t] += __shfl_xor(py[t], 16);
        py[t] += __shfl_xor(py[t], 32);
      }
      if (q == 0) *reinterpret_cast<v4f*>(yout + b * n + rg) = py + bp0;
    }
  }
}

// Forward layer tail, fused: the inverse slab pass of the spectral branch for
// the slab x of every channel of cell b (grid (x, b), C N threads), then
// h = W u + bias + s, uo = GELU(h) (or h) at the slab's points (C = 16: W u on
// the matrix cores, pointwise_mfma16), so that the spectral branch s never
// goes through global memory.  h and uo are stored
// only when non-null; lift.Fin set: u is the lifted input formed here; yout
// set (last layer): also the projection yout = sum_c Wp[c] uo[c] + bp; Tnext
// set: also the next layer's forward slab pass of uo into Tnext.
template <int N, int K, int C, bool CL>
__global__ __launch_bounds__(C * N) void k_fno_inv_slab_pointwise(
    const cx<float>* T, const float* __restrict__ u, LiftIn lift,
    const float* __restrict__ W, const float* __restrict__ bias, int act, float* __restrict__ h,
    float* __restrict__ uo, const float* __restrict__ Wp, const float* __restrict__ bp,
    float* __restrict__ yout, cx<float>* Tnext) {   // T and Tnext may alias
  using D = FnoDims<N, K>;
  constexpr int NT = C * N, LN = N + 1, n = D::n;
  // spectrum [C][N][K + 1] with an odd channel stride, so that lanes of
  // consecutive channels hit distinct banks
  constexpr int CS = N * (K + 1) + 1;
  constexpr int CBYTES = (int)sizeof(cx<float>) * C * CS;
  constexpr int RBYTES = (int)sizeof(float) * C * N * LN;
  __shared__ __align__(16) unsigned char raw[CBYTES > RBYTES ? CBYTES : RBYTES];
  cx<float>* const sp = reinterpret_cast<cx<float>*>(raw);
  auto lds = [sp](int c, int y, int col) -> cx<float>& { return sp[c * CS + y * (K + 1) + col]; };
  auto rl = reinterpret_cast<float(*)[N][LN]>(raw);            // [C][N][N + 1] branch s
  const int x = blockIdx.x;
  const int64_t b = blockIdx.y;
  for (int t = threadIdx.x; t < C * K; t += NT) {   // (channel, kz column) items
    // consecutive threads take consecutive entries of the layout
    const int c = CL ? t % C : t / K, col = CL ? t / C : t % K;
    cx<float> v[N];
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = {0.f, 0.f};
#pragma unroll
    for (int m = 0; m < D::KY; ++m) v[kidx<N, K>(m)] = T[tofs<N, K, C, CL>(b, c, x, m * K + col)];
    fft_line<N, +1>(v);
#pragma unroll
    for (int y = 0; y < N; ++y) lds(c, y, col) = v[y];
  }
  __syncthreads();
  const int c = threadIdx.x / N, i = threadIdx.x % N;   // thread (c, i): line y = i
  cx<float> v[N];
#pragma unroll
  for (int z = 0; z < N; ++z) v[z] = {0.f, 0.f};
#pragma unroll
  for (int kz = 0; kz < K; ++kz) v[kz] = lds(c, i, kz);
  fft_line<N, +1>(v);
  __syncthreads();                                // every read of the spectrum is done
#pragma unroll
  for (int z = 0; z < N; ++z) rl[c][i][z] = v[z].x;
  __syncthreads();
  if constexpr (C == 16) {
    pointwise_mfma16<N>(rl, x, b, u, lift, W, bias, act, h, uo, Wp, bp, yout, Tnext != nullptr);
  } else {
    for (int q = threadIdx.x; q < N * N; q += NT) {   // points (yy, zz) of the slab
      const int yy = q / N, zz = q % N;
      const int64_t r = (int64_t)x * N * N + q;
      float in[C];
      if (lift.Fin) {
        const float fv = lift.Fin[b * n + r];
#pragma unroll
        for (int k = 0; k < C; ++k) in[k] = lift.Wl[k] * fv + lift.bl[k];
      } else {
#pragma unroll
        for (int k = 0; k < C; ++k) in[k] = u[(b * C + k) * n + r];
      }
      float py = yout ? bp[0] : 0.f;
#pragma unroll
      for (int o = 0; o < C; ++o) {
        float acc = bias[o] + rl[o][yy][zz];
#pragma unroll
        for (int k = 0; k < C; ++k) acc += W[o * C + k] * in[k];
        if (h) h[(b * C + o) * n + r] = acc;
        const float out = act ? gelu(acc) : acc;
        if (uo) uo[(b * C + o) * n + r] = out;
        if (yout) py += Wp[o] * out;               // the projection sum_c Wp[c] u[c] + bp
        if (Tnext) rl[o][yy][zz] = out;            // this thread's own entries of s
      }
      if (yout) yout[b * n + r] = py;
    }
  }
  if (!Tnext) return;
  // the next layer's forward slab pass of the slab x of every channel, from
  // the outputs held in LDS; Tnext may be T itself (this block's slabs only)
  __syncthreads();
#pragma unroll
  for (int z = 0; z < N; ++z) v[z] = {rl[c][i][z], 0.f};   // thread (c, i): line y = i
  fft_line<N, -1>(v);
  __syncthreads();                                // every read of the outputs is done
#pragma unroll
  for (int kz = 0; kz < K; ++kz) lds(c, i, kz) = v[kz];
  __syncthreads();
  for (int t = threadIdx.x; t < C * K; t += NT) {   // (channel, kz column) items
    const int cc = CL ? t % C : t / K, col = CL ? t / C : t % K;
    cx<float> w[N];
#pragma unroll
    for (int y = 0; y < N; ++y) w[y] = lds(cc, y, col);
    fft_line<N, -1>(w);
#pragma unroll
    for (int m = 0; m < D::KY; ++m) Tnext[tofs<N, K, C, CL>(b, cc, x, m * K + col)] = w[kidx<N, K>(m)];
  }
}

// Inference, layer 0 at C = 16: the forward slab pass of the lifted input
// u0[c] = Wl[c] F~ + bl[c] of slab x of every channel of cell b, into the
// channel-last T (grid (x, b), 256 threads).  The pass is linear, so it is
// taken once, of F~ (wave 0: the z lines, then the y lines of the kept kz),
// and each channel's spectrum is Wl[c] S + bl[c] N^2 at ky = kz = 0 (the
// constant's unnormalised transform), written by every thread.
template <int N, int K, int C>
__global__ __launch_bounds__(256) void k_fno_lift_slab(LiftIn lift, cx<float>* __restrict__ T) {
  using D = FnoDims<N, K>;
  static_assert(N <= 64 && K <= 64, "one wave transforms the slab");
  __shared__ cx<float> lds[N][K + 1];
  __shared__ cx<float> S[D::PEN];
  const int x = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int t = threadIdx.x;
  if (t < N) {   // z line y = t
    const float* fs = lift.Fin + b * D::n + ((int64_t)x * N + t) * N;
    cx<float> v[N];
#pragma unroll
    for (int z = 0; z < N; ++z) v[z] = {fs[z], 0.f};
    fft_line<N, -1>(v);
#pragma unroll
    for (int kz = 0; kz < K; ++kz) lds[t][kz] = v[kz];
  }
  __syncthreads();
  if (t < K) {   // y line of kz = t
    cx<float> v[N];
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = lds[y][t];
    fft_line<N, -1>(v);
#pragma unroll
    for (int m = 0; m < D::KY; ++m) S[m * K + t] = v[kidx<N, K>(m)];
  }
  __syncthreads();
  cx<float>* Ts = T + tofs<N, K, C, true>(b, 0, x, 0);   // PEN x C contiguous values
  for (int e = t; e < D::PEN * C; e += 256) {
    const int c = e % C, pen = e / C;
    const cx<float> sv = S[pen];
    const float w = lift.Wl[c];
    Ts[e] = {fmaf(w, sv.x, pen == 0 ? lift.bl[c] * (float)(N * N) : 0.f), w * sv.y};
  }
}

// per-sample relative squared error and its gradient:
// loss_b = sum_r (y - t)^2 / (sum_r t^2 + eps);  dy = 2 (y - t) / (B (sum t^2 + eps)).
// Two passes over grid (RED_CHUNKS, B): sums of (y - t)^2 and t^2 over each
// chunk of a sample, then every block adds its sample's partials in a fixed
// order and writes dy over its chunk.  part: 2 RED_CHUNKS B doubles.
__global__ __launch_bounds__(256) void k_fno_loss_partial(const float* __restrict__ y,
                                                          const float* __restrict__ t, int n,
                                                          double* __restrict__ part) {
  __shared__ double red[2][256];
  const int b = blockIdx.y, j = blockIdx.x;
  const int chunk = n / RED_CHUNKS;
  const int64_t base = (int64_t)b * n + (int64_t)j * chunk;
  double se = 0.0, st = 0.0;
  for (int r = threadIdx.x; r < chunk; r += 256) {
    const double e = (double)y[base + r] - (double)t[base + r];
    const double tv = t[base + r];
    se += e * e;
    st += tv * tv;
  }
  red[0][threadIdx.x] = se;
  red[1][threadIdx.x] = st;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) part[((int64_t)b * RED_CHUNKS + j) * 2 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_fno_loss(const float* __restrict__ y,
                                                  const float* __restrict__ t, int B, int n,
                                                  const double* __restrict__ part,
                                                  float* __restrict__ dy,
                                                  double* __restrict__ loss_b) {
  const int b = blockIdx.y, j = blockIdx.x;
  const int chunk = n / RED_CHUNKS;
  double se = 0.0, st = 0.0;
  for (int k = 0; k < RED_CHUNKS; ++k) {
    se += part[((int64_t)b * RED_CHUNKS + k) * 2];
    st += part[((int64_t)b * RED_CHUNKS + k) * 2 + 1];
  }
  const double den = st + 1e-30;
  if (j == 0 && threadIdx.x == 0) loss_b[b] = se / den;
  const float sc = (float)(2.0 / ((double)B * den));
  const int64_t base = (int64_t)b * n + (int64_t)j * chunk;
  for (int r = threadIdx.x; r < chunk; r += 256) dy[base + r] = sc * (y[base + r] - t[base + r]);
}

// backward of the projection: du[b][c][r] = Wp[c] dy[b][r]
template <int C>
__global__ __launch_bounds__(256) void k_fno_proj_bwd(const float* __restrict__ dy, int B, int n,
                                                      const float* __restrict__ Wp,
                                                      float* __restrict__ du) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * n) return;
  const int64_t b = gid / n, r = gid % n;
  const float g = dy[gid];
#pragma unroll
  for (int c = 0; c < C; ++c) du[(b * C + c) * n + r] = Wp[c] * g;
}

// backward of a pointwise layer given du_out: dh = du_out * gelu'(h) (or du_out);
// du_in = W^T dh (spectral part added by the caller); writes dh
template <int C>
__global__ __launch_bounds__(256) void k_fno_pointwise_bwd(const float* __restrict__ duo,
                                                           const float* __restrict__ h, int B,
                                                           int n, const float* __restrict__ W,
                                                           int act, float* __restrict__ dh,
                                                           float* __restrict__ dui) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * n) return;
  const int64_t b = gid / n, r = gid % n;
  float g[C];
#pragma unroll
  for (int o = 0; o < C; ++o) {
    const float d = duo[(b * C + o) * n + r];
    g[o] = act ? d * gelu_d(h[(b * C + o) * n + r]) : d;
    dh[(b * C + o) * n + r] = g[o];
  }
#pragma unroll
  for (int i = 0; i < C; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int o = 0; o < C; ++o) acc += W[o * C + i] * g[o];
    dui[(b * C + i) * n + r] = acc;
  }
}

// The same at C = 16 with du_in = W^T dh on the matrix cores: one wave per 64
// points (grid B n / 256 blocks of four waves); lane (r, q) forms dh of
// channels 4 q .. 4 q + 3 at the four contiguous points 4 r .. 4 r + 3 (16-byte
// loads and stores), which are the B operand of four 16 x 16 x 16 products
// (tile t: points 4 r + t; A = W^T, lane (r, q) supplying W[4 q + j][r] at K
// step j), and ends with du_in of channels 4 q .. 4 q + 3 of the same points.
__global__ __launch_bounds__(256) void k_fno_pointwise_bwd16(const float* __restrict__ duo,
                                                             const float* __restrict__ h, int n,
                                                             const float* __restrict__ W, int act,
                                                             float* __restrict__ dh,
                                                             float* __restrict__ dui) {
  constexpr int C = 16;
  typedef float v4f __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const int64_t p = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64 + 4 * r;   // 64 | n
  const int64_t b = p / n, rr = p % n;
  float wa[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) wa[j] = W[(4 * q + j) * C + r];
  v4f g[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t o = (b * C + 4 * q + j) * n + rr;
    const v4f d = *reinterpret_cast<const v4f*>(duo + o);
    if (act) {
      const v4f hv = *reinterpret_cast<const v4f*>(h + o);
#pragma unroll
      for (int t = 0; t < 4; ++t) g[j][t] = d[t] * gelu_d(hv[t]);
    } else {
      g[j] = d;
    }
    *reinterpret_cast<v4f*>(dh + o) = g[j];
  }
  v4f acc[4];   // tile t: acc[t][v] = du_in of channel 4 q + v at point 4 r + t
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[j], g[j][t], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    *reinterpret_cast<v4f*>(dui + (b * C + 4 * q + v) * n + rr) =
        v4f{acc[0][v], acc[1][v], acc[2][v], acc[3][v]};
}

// Partial sums for the dense parameter gradients (fixed order, deterministic):
//   mode 0 (layer):  out[o*C+i] = sum dh[o] u[i], out[C*C + o] = sum dh[o]
//   mode 1 (lift):   out[c] = sum du0[c] Fin, out[C + c] = sum du0[c]
//   mode 2 (proj):   out[c] = sum dy u[c], out[C] = sum dy
// Block k sums the points [k npb, (k+1) npb) (npb a multiple of the tile, n
// too, so a tile never spans two cells): tiles of DG_TILE points of every
// channel of g (rows G) and a (rows A) are staged in LDS; each thread sums its
// values over a tile in FP32 and adds the tile sums in FP64.
// part[block][v], v < nvals.
constexpr int DG_TILE = 64;

template <int C>
__global__ __launch_bounds__(256) void k_fno_dense_partial(int mode, const float* __restrict__ a,
                                                           const float* __restrict__ g, int B,
                                                           int n, int npb,
                                                           float* __restrict__ part) {
  constexpr int NV = C * C + C, LT = DG_TILE + 4;   // rows 16-byte aligned, banks staggered
  static_assert(NV <= 512, "two values per thread");
  __shared__ __align__(16) float G[C][LT];
  __shared__ __align__(16) float A[C][LT];
  const int64_t total = (int64_t)B * n;
  const int nvals = mode == 0 ? NV : (mode == 1 ? 2 * C : C + 1);
  const int gr = mode == 2 ? 1 : C;               // rows of G and A in this mode
  const int ar = mode == 1 ? 1 : C;
  // the rows of this thread's values (-1: factor 1)
  int gi[2], ai[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int v = threadIdx.x + 256 * k;
    if (mode == 0) {
      gi[k] = v < C * C ? v / C : v - C * C;
      ai[k] = v < C * C ? v % C : -1;
    } else if (mode == 1) {
      gi[k] = v < C ? v : v - C;
      ai[k] = v < C ? 0 : -1;
    } else {
      gi[k] = 0;
      ai[k] = v < C ? v : -1;
    }
    if (v >= nvals) gi[k] = -1;
  }
  double acc[2] = {0.0, 0.0};
  const int64_t p0 = (int64_t)blockIdx.x * npb;
  const int64_t p1 = min(p0 + (int64_t)npb, total);
  // this thread's share of a tile: entries e = threadIdx.x + 256 q of the
  // (gr + ar) x DG_TILE rows, loaded one tile ahead
  constexpr int PRE = (2 * C * DG_TILE + 255) / 256;
  float pre[PRE];
  auto load_tile = [&](int64_t t0) {
    const int64_t b = t0 / n, r0 = t0 % n;
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int row = e / DG_TILE, p = e % DG_TILE;
      float v = 0.f;
      if (row < gr + ar && t0 + p < total) {
        if (row < gr) {
          // mode 2: G row 0 = dy[b][r]; otherwise G rows = g[b][c][r]
          v = g[mode == 2 ? t0 + p : (b * C + row) * n + r0 + p];
        } else {
          v = a[mode == 1 ? t0 + p : (b * C + (row - gr)) * n + r0 + p];
        }
      }
      pre[q] = v;
    }
  };
  if (p0 < p1) load_tile(p0);
  for (int64_t t0 = p0; t0 < p1; t0 += DG_TILE) {
    __syncthreads();                              // the previous tile is consumed
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int row = e / DG_TILE, p = e % DG_TILE;
      if (row < gr) G[row][p] = pre[q];
      else if (row < gr + ar) A[row - gr][p] = pre[q];
    }
    __syncthreads();
    if (t0 + DG_TILE < p1) load_tile(t0 + DG_TILE);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (gi[k] < 0) continue;
      const float4* gp = reinterpret_cast<const float4*>(G[gi[k]]);
      float s = 0.f;
      if (ai[k] >= 0) {
        const float4* ap = reinterpret_cast<const float4*>(A[ai[k]]);
#pragma unroll
        for (int p = 0; p < DG_TILE / 4; ++p) {
          const float4 x = gp[p], y = ap[p];
          s += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
        }
      } else {
#pragma unroll
        for (int p = 0; p < DG_TILE / 4; ++p) {
          const float4 x = gp[p];
          s += (x.x + x.y) + (x.z + x.w);
        }
      }
      acc[k] += (double)s;
    }
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int v = threadIdx.x + 256 * k;
    if (v < nvals) part[(int64_t)blockIdx.x * NV + v] = (float)acc[k];
  }
}

// Mode 0 at C = 16 on the matrix cores: out[o][i] = sum dh[o] u[i] as 16 x 16
// x 4 products over the block's points (operand layout as in the mode
// mixing: lane (r, q) loads points 4 q .. 4 q + 3 of a 16-point group of row r
// of dh and of u, one 16-byte load each, and K step s takes point 4 q + s;
// wave w takes the groups w, w + 4, ...), FP32 sums over a wave's points and
// FP64 over the block's four waves; out[C C + o] = sum dh[o] from the same
// loads.  part[block][v] as k_fno_dense_partial.
__global__ __launch_bounds__(256) void k_fno_dense_mfma16(const float* __restrict__ a,
                                                          const float* __restrict__ g, int n,
                                                          int npb, int64_t total,
                                                          float* __restrict__ part) {
  constexpr int C = 16, NV = C * C + C;
  typedef float v4f __attribute__((ext_vector_type(4)));
  __shared__ float red[4][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int64_t p0 = (int64_t)blockIdx.x * npb;
  const int64_t p1 = min(p0 + (int64_t)npb, total);
  const int ng = p1 > p0 ? (int)((p1 - p0) / 16) : 0;   // 16 divides npb and n
  v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
  float bs = 0.f;
  for (int gi = wv; gi < ng; gi += 4) {   // uniform per wave
    const int64_t pt = p0 + 16 * gi + 4 * q;
    const int64_t b = pt / n, rr = pt % n;
    const v4f gv = *reinterpret_cast<const v4f*>(g + (b * C + r) * n + rr);
    const v4f av = *reinterpret_cast<const v4f*>(a + (b * C + r) * n + rr);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[k], av[k], acc, 0, 0, 0);
    bs += (gv[0] + gv[1]) + (gv[2] + gv[3]);
  }
  // lane (r, q): acc[v] = out[4 q + v][r]; bs: row r over the lane's points
  bs += __shfl_xor(bs, 16);
  bs += __shfl_xor(bs, 32);
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wv][(4 * q + v) * C + r] = acc[v];
  if (q == 0) red[wv][C * C + r] = bs;
  __syncthreads();
  for (int v = threadIdx.x; v < NV; v += 256) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) sum += (double)red[w][v];
    part[(int64_t)blockIdx.x * NV + v] = (float)sum;
  }
}

// out[v] = sum_k part[k][v] (FP64, fixed order); one block per value
template <int C>
__global__ __launch_bounds__(256) void k_fno_dense_final(const float* __restrict__ part,
                                                         int nblocks, float* __restrict__ out) {
  constexpr int NV = C * C + C;
  __shared__ double red[256];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += 256) acc += part[(int64_t)k * NV + v];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = (float)red[0];
}

// Adam (bias-corrected), FP32 parameters and moments
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              int64_t np, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// input scale c0 = (2 pi)^{3/2}
constexpr double kInputScale = 15.749609945653303;

// F~ = c0 F / mass (FP64 cell in the batch layout -> FP32), mass[b] = h^3 sum F.
// Two passes over grid (RED_CHUNKS, B): partial sums of F over each chunk of
// a cell, then every block adds the partials of its cell in a fixed order and
// scales its chunk (deterministic; each cell is spread over RED_CHUNKS blocks).
__global__ __launch_bounds__(256) void k_fno_mass_partial(const double* __restrict__ f,
                                                          const int64_t* __restrict__ off,
                                                          int64_t cell0, int n,
                                                          double* __restrict__ part) {
  __shared__ double red[256];
  const int b = blockIdx.y, j = blockIdx.x;
  const int chunk = n / RED_CHUNKS;
  const double* fc = f + off[cell0 + b] + (int64_t)j * chunk;
  double acc = 0.0;
  for (int r = threadIdx.x; r < chunk; r += 256) acc += fc[r];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)b * RED_CHUNKS + j] = red[0];
}

__global__ __launch_bounds__(256) void k_fno_normalize(const double* __restrict__ f,
                                                       const int64_t* __restrict__ off,
                                                       int64_t cell0, int n, double hd,
                                                       const double* __restrict__ part,
                                                       float* __restrict__ Fin,
                                                       double* __restrict__ mass) {
  const int b = blockIdx.y, j = blockIdx.x;
  const int chunk = n / RED_CHUNKS;
  double sum = 0.0;
  for (int k = 0; k < RED_CHUNKS; ++k) sum += part[(int64_t)b * RED_CHUNKS + k];
  const double ms = hd * sum;
  if (j == 0 && threadIdx.x == 0) mass[b] = ms;
  const double inv = ms > 0.0 ? kInputScale / ms : 0.0;
  const double* fc = f + off[cell0 + b] + (int64_t)j * chunk;
  float* out = Fin + (int64_t)b * n + (int64_t)j * chunk;
  for (int r = threadIdx.x; r < chunk; r += 256) out[r] = (float)(fc[r] * inv);
}

// target = c0^2 Q / mass^2 (FP64 cell in the batch layout -> FP32)
__global__ __launch_bounds__(256) void k_fno_target(const double* __restrict__ Q,
                                                    const int64_t* __restrict__ off, int64_t cell0,
                                                    int n, int B, const double* __restrict__ mass,
                                                    float* __restrict__ t) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * n) return;
  const int b = (int)(gid / n), r = (int)(gid % n);
  const double m = mass[b];
  t[gid] = m > 0.0 ? (float)(Q[off[cell0 + b] + r] * (kInputScale * kInputScale) / (m * m)) : 0.f;
}

// Q = mass^2 y / c0^2 (FP32 -> FP64 cell in the batch layout)
__global__ __launch_bounds__(256) void k_fno_denormalize(const float* __restrict__ y,
                                                         const double* __restrict__ mass,
                                                         const int64_t* __restrict__ off,
                                                         int64_t cell0, int n, int B,
                                                         double* __restrict__ Q) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * n) return;
  const int b = (int)(gid / n), r = (int)(gid % n);
  Q[off[cell0 + b] + r] = mass[b] * mass[b] * (double)y[gid] / (kInputScale * kInputScale);
}

// ---------------------------------------------------------------------------
// launchers (sizes fixed per instantiation)
// ---------------------------------------------------------------------------
template <int C>
static unsigned mix_blocks(int B, int NM) {
  const int64_t nt = (int64_t)((B + MIX_CELLS - 1) / MIX_CELLS) * NM * C;
  return (unsigned)((nt + 255) / 256);
}

// mode mixing (forward, or the adjoint with conj R transposed): on the matrix
// cores at C = 16, on the vector ALU otherwise
template <int C>
static void launch_mix(const cx<float>* R, const cx<float>* X, int B, int NM, int adjoint,
                       float scale, cx<float>* Y, hipStream_t st) {
  if constexpr (C == 16) {
    const int64_t waves = (int64_t)((B + MIX_MFMA_CELLS - 1) / MIX_MFMA_CELLS) * NM;
    hipLaunchKernelGGL(k_fno_mix_mfma16, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, R,
                       X, B, NM, adjoint, scale, Y);
  } else {
    hipLaunchKernelGGL((k_fno_mix2<C>), dim3(mix_blocks<C>(B, NM)), dim3(256), 0, st, R, X, B,
                       NM, adjoint, scale, Y);
  }
}

template <int N, int K, int C>
struct FnoOps {
  using D = FnoDims<N, K>;
  static hipError_t fwd_transform(const float* u, int nsc, cx<float>* T, cx<float>* Uh,
                                  hipStream_t st, LiftIn lift = LiftIn()) {
    const int64_t nslab = (int64_t)nsc * N;
    constexpr int SB = slabs_per_block<N>(), TP = pens_per_block<C>();
    hipLaunchKernelGGL((k_fno_fwd_slab<N, K>), dim3((unsigned)((nslab + SB - 1) / SB)), dim3(256),
                       0, st, u, T, nslab, lift, C);
    hipLaunchKernelGGL((k_fno_fwd_x<N, K, C>), dim3((D::PEN + TP - 1) / TP, (unsigned)(nsc / C)),
                       dim3(256), 0, st, T, Uh);
    return hipGetLastError();
  }
  // inference at C = 16 (channel-last T): the lifted input's forward slab
  // pass, and the x transforms with the mode mixing, fused
  static hipError_t lift_slab_cl(const LiftIn& lift, int B, cx<float>* T, hipStream_t st) {
    hipLaunchKernelGGL((k_fno_lift_slab<N, K, C>), dim3(N, (unsigned)B), dim3(256), 0, st, lift, T);
    return hipGetLastError();
  }
  static hipError_t xmix_cl(cx<float>* T, int B, const cx<float>* R, float scale, hipStream_t st) {
    hipLaunchKernelGGL((k_fno_xmix16<N, K>), dim3(D::PEN, (unsigned)((B + 15) / 16)), dim3(256), 0,
                       st, T, B, R, scale);
    return hipGetLastError();
  }
  static hipError_t fwd_x_pass(const cx<float>* T, int nsc, cx<float>* Uh, hipStream_t st) {
    constexpr int TP = pens_per_block<C>();
    hipLaunchKernelGGL((k_fno_fwd_x<N, K, C>), dim3((D::PEN + TP - 1) / TP, (unsigned)(nsc / C)),
                       dim3(256), 0, st, T, Uh);
    return hipGetLastError();
  }
  static hipError_t inv_x_pass(const cx<float>* V, int nsc, cx<float>* T, hipStream_t st) {
    constexpr int TP = pens_per_block<C>();
    hipLaunchKernelGGL((k_fno_inv_x<N, K, C>), dim3((D::PEN + TP - 1) / TP, (unsigned)(nsc / C)),
                       dim3(256), 0, st, V, T);
    return hipGetLastError();
  }
  static hipError_t inv_transform(const cx<float>* V, int nsc, cx<float>* T, float* out,
                                  int accumulate, hipStream_t st) {
    const int64_t nslab = (int64_t)nsc * N;
    constexpr int SB = slabs_per_block<N>(), TP = pens_per_block<C>();
    hipLaunchKernelGGL((k_fno_inv_x<N, K, C>), dim3((D::PEN + TP - 1) / TP, (unsigned)(nsc / C)),
                       dim3(256), 0, st, V, T);
    hipLaunchKernelGGL((k_fno_inv_slab<N, K>), dim3((unsigned)((nslab + SB - 1) / SB)), dim3(256),
                       0, st, T, out, nslab, accumulate);
    return hipGetLastError();
  }
};

template <int N, int K, int C>
static hipError_t fno_forward_t(const FnoArgs& a, hipStream_t st) {
  using D = FnoDims<N, K>;
  using O = FnoOps<N, K, C>;
  const int B = a.B;
  const int n = D::n;
  const int64_t bn = (int64_t)B * n;
  const unsigned gb = (unsigned)((bn + 255) / 256);
  // training keeps every activation for the backward pass; inference forms the
  // lifted input where it is read and stores neither u0 nor the last layer's u
  const bool keep = a.store_h;
  LiftIn lift;
  if (keep) {
    hipLaunchKernelGGL((k_fno_lift<C>), dim3(gb), dim3(256), 0, st, a.Fin, B, n, a.Wl, a.bl,
                       a.u[0]);
  } else {
    lift.Fin = a.Fin;
    lift.Wl = a.Wl;
    lift.bl = a.bl;
  }
  for (int l = 0; l < a.L; ++l) {
    const LiftIn li = l == 0 ? lift : LiftIn();
    const bool last = l + 1 == a.L;
    // the slab pass of layers l > 0 ran in the previous layer's last kernel.
    // Inference at C = 16 runs the x transforms and the mixing fused on the
    // channel-last T; training, which stores the kept modes Uh for the weight
    // gradient, and the other channel counts run them as separate kernels on
    // the channel-first T
    float* hl = keep ? a.h[l] : nullptr;
    float* uo = keep || !last ? a.u[l + 1] : nullptr;
    float* yo = last ? a.y : nullptr;
    cx<float>* Tn = last ? nullptr : a.T;
    hipError_t e = hipSuccess;
    bool fused = false;
    if constexpr (C == 16) {
      if (!keep) {
        e = l == 0 ? O::lift_slab_cl(li, B, a.T, st) : hipSuccess;
        if (e != hipSuccess) return e;
        e = O::xmix_cl(a.T, B, a.R[l], 1.f / (float)n, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_fno_inv_slab_pointwise<N, K, C, true>), dim3(N, (unsigned)B),
                           dim3(C * N), 0, st, a.T, a.u[l], li, a.W[l], a.bias[l], last ? 0 : 1,
                           hl, uo, a.Wp, a.bp, yo, Tn);
        fused = true;
      }
    }
    if (!fused) {
      e = l == 0 ? O::fwd_transform(a.u[l], B * C, a.T, a.Uh[l], st, li)
                 : O::fwd_x_pass(a.T, B * C, a.Uh[l], st);
      if (e != hipSuccess) return e;
      launch_mix<C>(a.R[l], a.Uh[l], B, D::NM, 0, 1.f / (float)n, a.V, st);
      e = O::inv_x_pass(a.V, B * C, a.T, st);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_fno_inv_slab_pointwise<N, K, C, false>), dim3(N, (unsigned)B),
                         dim3(C * N), 0, st, a.T, a.u[l], li, a.W[l], a.bias[l], last ? 0 : 1, hl,
                         uo, a.Wp, a.bp, yo, Tn);
    }
  }
  return hipGetLastError();
}

template <int C>
static hipError_t dense_grad(int mode, const float* act, const float* g, int B, int n, float* part,
                             int part_blocks, float* out, hipStream_t st) {
  const int64_t total = (int64_t)B * n;
  // points per block: a whole number of tiles
  const int64_t per = (total + part_blocks - 1) / part_blocks;
  const int npb = (int)((per + DG_TILE - 1) / DG_TILE * DG_TILE);
  bool done = false;
  if constexpr (C == 16) {
    if (mode == 0) {   // the layers' weight gradients, on the matrix cores
      hipLaunchKernelGGL(k_fno_dense_mfma16, dim3(part_blocks), dim3(256), 0, st, act, g, n, npb,
                         total, part);
      done = true;
    }
  }
  if (!done) {
    hipLaunchKernelGGL((k_fno_dense_partial<C>), dim3(part_blocks), dim3(256), 0, st, mode, act,
                       g, B, n, npb, part);
  }
  const int nvals = mode == 0 ? C * C + C : (mode == 1 ? 2 * C : C + 1);
  hipLaunchKernelGGL((k_fno_dense_final<C>), dim3(nvals), dim3(256), 0, st, part, part_blocks,
                     out);
  return hipGetLastError();
}

template <int N, int K, int C>
static hipError_t fno_backward_t(const FnoArgs& args, hipStream_t st) {
  FnoArgs a = args;   // du / du2 swap roles layer by layer
  using D = FnoDims<N, K>;
  using O = FnoOps<N, K, C>;
  const int B = a.B;
  const int n = D::n;
  const int64_t bn = (int64_t)B * n;
  const unsigned gb = (unsigned)((bn + 255) / 256);
  hipError_t e;
  // loss and projection
  {
    // the dense-gradient scratch is free until the first dense_grad below
    double* lp = reinterpret_cast<double*>(a.part);
    const dim3 grid(RED_CHUNKS, (unsigned)B);
    hipLaunchKernelGGL(k_fno_loss_partial, grid, dim3(256), 0, st, a.y, a.target, n, lp);
    hipLaunchKernelGGL(k_fno_loss, grid, dim3(256), 0, st, a.y, a.target, B, n, lp, a.dy,
                       a.loss_b);
  }
  e = dense_grad<C>(2, a.u[a.L], a.dy, B, n, a.part, a.part_blocks, a.gWp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fno_proj_bwd<C>), dim3(gb), dim3(256), 0, st, a.dy, B, n, a.Wp, a.du);
  for (int l = a.L - 1; l >= 0; --l) {
    // dh (into a.dh), pointwise part of du_in (into a.du2)
    if constexpr (C == 16) {
      static_assert(D::n % 256 == 0, "one wave per 64 points of a cell");
      hipLaunchKernelGGL(k_fno_pointwise_bwd16, dim3((unsigned)(bn / 256)), dim3(256), 0, st, a.du,
                         a.h[l], n, a.W[l], l + 1 < a.L ? 1 : 0, a.dh, a.du2);
    } else {
      hipLaunchKernelGGL((k_fno_pointwise_bwd<C>), dim3(gb), dim3(256), 0, st, a.du, a.h[l], B,
                         n, a.W[l], l + 1 < a.L ? 1 : 0, a.dh, a.du2);
    }
    e = dense_grad<C>(0, a.u[l], a.dh, B, n, a.part, a.part_blocks, a.gW[l], st);
    if (e != hipSuccess) return e;
    // spectral part: Gv = truncated DFT(dh); dR = sum_b Gv conj(Uh); Gu = conj(R)^T Gv
    e = O::fwd_transform(a.dh, B * C, a.T, a.V, st);
    if (e != hipSuccess) return e;
    const int64_t nmc = (int64_t)D::NM * C;
    hipLaunchKernelGGL((k_fno_dR<C>), dim3((unsigned)((nmc + 255) / 256)), dim3(256), 0, st, a.V,
                       a.Uh[l], B, D::NM, 1.f / (float)n, a.gR[l]);
    launch_mix<C>(a.R[l], a.V, B, D::NM, 1, 1.f / (float)n, a.V2, st);
    // du_in = pointwise part + Re IDFT(scatter(Gu))
    e = O::inv_transform(a.V2, B * C, a.T, a.du2, 1, st);
    if (e != hipSuccess) return e;
    float* tmp = a.du;
    a.du = a.du2;
    a.du2 = tmp;
  }
  // lift: du now holds the gradient of u0
  e = dense_grad<C>(1, a.Fin, a.du, B, n, a.part, a.part_blocks, a.gWl, st);
  return e;
}

hipError_t fno_forward(const FnoArgs& a, hipStream_t st) {
  if (a.N == 32 && a.K == 12 && a.C == 16) return fno_forward_t<32, 12, 16>(a, st);
  if (a.N == 8 && a.K == 2 && a.C == 4) return fno_forward_t<8, 2, 4>(a, st);
  if (a.N == 16 && a.K == 6 && a.C == 8) return fno_forward_t<16, 6, 8>(a, st);
  return hipErrorInvalidValue;
}

hipError_t fno_backward(const FnoArgs& a, hipStream_t st) {
  if (a.N == 32 && a.K == 12 && a.C == 16) return fno_backward_t<32, 12, 16>(a, st);
  if (a.N == 8 && a.K == 2 && a.C == 4) return fno_backward_t<8, 2, 4>(a, st);
  if (a.N == 16 && a.K == 6 && a.C == 8) return fno_backward_t<16, 6, 8>(a, st);
  return hipErrorInvalidValue;
}

bool fno_supported(int N, int K, int C) {
  return (N == 32 && K == 12 && C == 16) || (N == 8 && K == 2 && C == 4) ||
         (N == 16 && K == 6 && C == 8);
}

hipError_t fno_adam(float* p, const float* g, float* m, float* v, int64_t np, float lr, float b1,
                    float b2, float eps, int step, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, p, g, m, v, np,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t fno_normalize(const double* f, const int64_t* off, int64_t cell0, int n, double hd,
                         int B, double* part, float* Fin, double* mass, hipStream_t st) {
  if (n % RED_CHUNKS) return hipErrorInvalidValue;
  const dim3 grid(RED_CHUNKS, (unsigned)B);
  hipLaunchKernelGGL(k_fno_mass_partial, grid, dim3(256), 0, st, f, off, cell0, n, part);
  hipLaunchKernelGGL(k_fno_normalize, grid, dim3(256), 0, st, f, off, cell0, n, hd, part, Fin,
                     mass);
  return hipGetLastError();
}

hipError_t fno_target(const double* Q, const int64_t* off, int64_t cell0, int n, int B,
                      const double* mass, float* t, hipStream_t st) {
  const int64_t bn = (int64_t)B * n;
  hipLaunchKernelGGL(k_fno_target, dim3((unsigned)((bn + 255) / 256)), dim3(256), 0, st, Q, off,
                     cell0, n, B, mass, t);
  return hipGetLastError();
}

hipError_t fno_denormalize(const float* y, const double* mass, const int64_t* off, int64_t cell0,
                           int n, int B, double* Q, hipStream_t st) {
  const int64_t bn = (int64_t)B * n;
  hipLaunchKernelGGL(k_fno_denormalize, dim3((unsigned)((bn + 255) / 256)), dim3(256), 0, st, y,
                     mass, off, cell0, n, B, Q);
  return hipGetLastError();
}

}  // namespace efm

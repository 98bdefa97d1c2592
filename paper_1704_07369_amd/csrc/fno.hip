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
// 2K kx); inverse = the same passes backwards with zero padding.
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

// ---------------------------------------------------------------------------
// truncated forward transform, slab pass: real u[s][x][y][z] -> T[s][x][ky][kz]
// one block per (s, x) slab, N threads
// ---------------------------------------------------------------------------
template <int N, int K>
__global__ __launch_bounds__(N) void k_fno_fwd_slab(const float* __restrict__ u,
                                                    cx<float>* __restrict__ T) {
  using D = FnoDims<N, K>;
  __shared__ cx<float> lds[N][K + 1];
  const int i = threadIdx.x;
  const int64_t slab = blockIdx.x;                // s * N + x
  const float* us = u + slab * N * N;
  cx<float> v[N];
#pragma unroll
  for (int z = 0; z < N; ++z) v[z] = {us[i * N + z], 0.f};   // thread i: line y = i
  fft_line<N, -1>(v);
#pragma unroll
  for (int kz = 0; kz < K; ++kz) lds[i][kz] = v[kz];
  __syncthreads();
  if (i < K) {                                    // thread i: kz column i
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = lds[y][i];
    fft_line<N, -1>(v);
    cx<float>* Ts = T + slab * D::PEN;
#pragma unroll
    for (int m = 0; m < D::KY; ++m) Ts[m * K + i] = v[kidx<N, K>(m)];
  }
}

// truncated forward transform, x pass: T[s][x][pen] -> Uh[b][mode][c] (s = b*C + c)
template <int N, int K, int C>
__global__ __launch_bounds__(64) void k_fno_fwd_x(const cx<float>* __restrict__ T, int nsc,
                                                  cx<float>* __restrict__ Uh) {
  using D = FnoDims<N, K>;
  const int64_t gid = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (gid >= (int64_t)nsc * D::PEN) return;
  const int s = (int)(gid / D::PEN), pen = (int)(gid % D::PEN);
  const cx<float>* Ts = T + (int64_t)s * N * D::PEN + pen;
  cx<float> v[N];
#pragma unroll
  for (int x = 0; x < N; ++x) v[x] = Ts[(int64_t)x * D::PEN];
  fft_line<N, -1>(v);
  const int b = s / C, c = s % C;
#pragma unroll
  for (int mx = 0; mx < D::KY; ++mx) {
    const int mode = mx * D::PEN + pen;
    Uh[((int64_t)b * D::NM + mode) * C + c] = v[kidx<N, K>(mx)];
  }
}

// truncated inverse transform, x pass: V[b][mode][c] -> T[s][x][pen]
template <int N, int K, int C>
__global__ __launch_bounds__(64) void k_fno_inv_x(const cx<float>* __restrict__ V, int nsc,
                                                  cx<float>* __restrict__ T) {
  using D = FnoDims<N, K>;
  const int64_t gid = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (gid >= (int64_t)nsc * D::PEN) return;
  const int s = (int)(gid / D::PEN), pen = (int)(gid % D::PEN);
  const int b = s / C, c = s % C;
  cx<float> v[N];
#pragma unroll
  for (int x = 0; x < N; ++x) v[x] = {0.f, 0.f};
#pragma unroll
  for (int mx = 0; mx < D::KY; ++mx)
    v[kidx<N, K>(mx)] = V[((int64_t)b * D::NM + mx * D::PEN + pen) * C + c];
  fft_line<N, +1>(v);
  cx<float>* Ts = T + (int64_t)s * N * D::PEN + pen;
#pragma unroll
  for (int x = 0; x < N; ++x) Ts[(int64_t)x * D::PEN] = v[x];
}

// truncated inverse transform, slab pass: T[s][x][ky][kz] -> out[s][x][y][z] = Re(...)
// (accumulate != 0: out += result)
template <int N, int K>
__global__ __launch_bounds__(N) void k_fno_inv_slab(const cx<float>* __restrict__ T,
                                                    float* __restrict__ out, int accumulate) {
  using D = FnoDims<N, K>;
  __shared__ cx<float> lds[N][K + 1];
  const int i = threadIdx.x;
  const int64_t slab = blockIdx.x;
  const cx<float>* Ts = T + slab * D::PEN;
  cx<float> v[N];
  if (i < K) {                                    // thread i: kz column i
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = {0.f, 0.f};
#pragma unroll
    for (int m = 0; m < D::KY; ++m) v[kidx<N, K>(m)] = Ts[m * K + i];
    fft_line<N, +1>(v);
#pragma unroll
    for (int y = 0; y < N; ++y) lds[y][i] = v[y];
  }
  __syncthreads();
#pragma unroll
  for (int z = 0; z < N; ++z) v[z] = {0.f, 0.f};
#pragma unroll
  for (int kz = 0; kz < K; ++kz) v[kz] = lds[i][kz];        // thread i: line y = i
  fft_line<N, +1>(v);
  float* os = out + slab * N * N;
#pragma unroll
  for (int z = 0; z < N; ++z) {
    if (accumulate) os[i * N + z] += v[z].x;
    else os[i * N + z] = v[z].x;
  }
}

// ---------------------------------------------------------------------------
// mode mixing.  forward: Y[b][m][o] = scale sum_i R[m][i][o] X[b][m][i]
// adjoint:              Y[b][m][i] = scale sum_o conj(R[m][i][o]) X[b][m][o]
// one thread per (b, m, output channel)
// ---------------------------------------------------------------------------
template <int C>
__global__ __launch_bounds__(256) void k_fno_mix2(const cx<float>* __restrict__ R,
                                                  const cx<float>* __restrict__ X, int B, int NM,
                                                  int adjoint, float scale,
                                                  cx<float>* __restrict__ Y) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * NM * C) return;
  const int o = (int)(gid % C);
  const int64_t bm = gid / C;
  const int m = (int)(bm % NM);
  const cx<float>* x = X + bm * C;
  const cx<float>* Rm = R + (int64_t)m * C * C;
  cx<float> acc = {0.f, 0.f};
  if (!adjoint) {
#pragma unroll
    for (int i = 0; i < C; ++i) acc = cadd(acc, cmul(Rm[i * C + o], x[i]));
  } else {
#pragma unroll
    for (int oo = 0; oo < C; ++oo) {
      const cx<float> r = Rm[o * C + oo];        // R[m][i = o][oo]
      acc = cadd(acc, cmul({r.x, -r.y}, x[oo]));
    }
  }
  Y[gid] = {scale * acc.x, scale * acc.y};
}

// dR[m][i][o] = scale sum_b G[b][m][o] conj(U[b][m][i]); one thread per (m, i, o)
template <int C>
__global__ __launch_bounds__(256) void k_fno_dR(const cx<float>* __restrict__ G,
                                                const cx<float>* __restrict__ U, int B, int NM,
                                                float scale, cx<float>* __restrict__ dR) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)NM * C * C) return;
  const int o = (int)(gid % C);
  const int i = (int)((gid / C) % C);
  const int64_t m = gid / (C * C);
  cx<float> acc = {0.f, 0.f};
  for (int b = 0; b < B; ++b) {
    const cx<float> g = G[((int64_t)b * NM + m) * C + o];
    const cx<float> uu = U[((int64_t)b * NM + m) * C + i];
    acc = cadd(acc, cmul(g, {uu.x, -uu.y}));
  }
  dR[gid] = {scale * acc.x, scale * acc.y};
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

// h[b][o][r] = sum_i W[o][i] u[b][i][r] + bias[o] + s[b][o][r]; uo = gelu(h) or h
template <int C>
__global__ __launch_bounds__(256) void k_fno_pointwise(const float* __restrict__ u,
                                                       const float* __restrict__ s, int B, int n,
                                                       const float* __restrict__ W,
                                                       const float* __restrict__ bias,
                                                       int act, float* __restrict__ h,
                                                       float* __restrict__ uo) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * n) return;
  const int64_t b = gid / n, r = gid % n;
  float in[C];
#pragma unroll
  for (int i = 0; i < C; ++i) in[i] = u[(b * C + i) * n + r];
#pragma unroll
  for (int o = 0; o < C; ++o) {
    float acc = bias[o] + s[(b * C + o) * n + r];
#pragma unroll
    for (int i = 0; i < C; ++i) acc += W[o * C + i] * in[i];
    h[(b * C + o) * n + r] = acc;
    uo[(b * C + o) * n + r] = act ? gelu(acc) : acc;
  }
}

// y[b][r] = sum_c Wp[c] u[b][c][r] + bp
template <int C>
__global__ __launch_bounds__(256) void k_fno_proj(const float* __restrict__ u, int B, int n,
                                                  const float* __restrict__ Wp,
                                                  const float* __restrict__ bp,
                                                  float* __restrict__ y) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)B * n) return;
  const int64_t b = gid / n, r = gid % n;
  float acc = bp[0];
#pragma unroll
  for (int c = 0; c < C; ++c) acc += Wp[c] * u[(b * C + c) * n + r];
  y[gid] = acc;
}

// per-sample relative squared error and its gradient:
// loss_b = sum_r (y - t)^2 / (sum_r t^2 + eps);  dy = 2 (y - t) / (B (sum t^2 + eps))
// one block per sample
__global__ __launch_bounds__(256) void k_fno_loss(const float* __restrict__ y,
                                                  const float* __restrict__ t, int B, int n,
                                                  float* __restrict__ dy, double* __restrict__ loss_b) {
  __shared__ double red[2][256];
  const int b = blockIdx.x;
  double se = 0.0, st = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double e = (double)y[(int64_t)b * n + r] - (double)t[(int64_t)b * n + r];
    const double tv = t[(int64_t)b * n + r];
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
  const double den = red[1][0] + 1e-30;
  if (threadIdx.x == 0) loss_b[b] = red[0][0] / den;
  const float sc = (float)(2.0 / ((double)B * den));
  for (int r = threadIdx.x; r < n; r += 256)
    dy[(int64_t)b * n + r] = sc * (y[(int64_t)b * n + r] - t[(int64_t)b * n + r]);
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

// Partial sums for the dense parameter gradients (fixed order, deterministic):
//   mode 0 (layer):  out[o*C+i] = sum dh[o] u[i], out[C*C + o] = sum dh[o]
//   mode 1 (lift):   out[c] = sum du0[c] Fin, out[C + c] = sum du0[c]
//   mode 2 (proj):   out[c] = sum dy u[c], out[C] = sum dy
// grid: blocks over points; each block writes nvals partials to part[block]
template <int C>
__global__ __launch_bounds__(256) void k_fno_dense_partial(int mode, const float* __restrict__ a,
                                                           const float* __restrict__ g, int B,
                                                           int n, int npb,
                                                           float* __restrict__ part) {
  constexpr int NV = C * C + C;
  __shared__ float red[256];
  const int64_t p0 = (int64_t)blockIdx.x * npb;
  const int64_t total = (int64_t)B * n;
  const int nvals = mode == 0 ? NV : (mode == 1 ? 2 * C : C + 1);
  for (int v = 0; v < nvals; ++v) {
    float acc = 0.f;
    for (int64_t q = p0 + threadIdx.x; q < p0 + npb && q < total; q += 256) {
      const int64_t b = q / n, r = q % n;
      float x;
      if (mode == 0) {
        if (v < C * C) {
          const int o = v / C, i = v % C;
          x = g[(b * C + o) * n + r] * a[(b * C + i) * n + r];
        } else {
          x = g[(b * C + (v - C * C)) * n + r];
        }
      } else if (mode == 1) {
        const int c = v % C;
        x = g[(b * C + c) * n + r] * (v < C ? a[q] : 1.f);
      } else {
        x = v < C ? g[q] * a[(b * C + v) * n + r] : g[q];
      }
      acc += x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * NV + v] = red[0];
    __syncthreads();
  }
}

template <int C>
__global__ void k_fno_dense_final(const float* __restrict__ part, int nblocks, int nvals,
                                  float* __restrict__ out) {
  constexpr int NV = C * C + C;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvals) return;
  double acc = 0.0;
  for (int k = 0; k < nblocks; ++k) acc += part[(int64_t)k * NV + v];
  out[v] = (float)acc;
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

// F~ = c0 F / mass (FP64 cell in the batch layout -> FP32), mass[b] = h^3 sum F
__global__ __launch_bounds__(256) void k_fno_normalize(const double* __restrict__ f,
                                                       const int64_t* __restrict__ off,
                                                       int64_t cell0, int n, double hd,
                                                       float* __restrict__ Fin,
                                                       double* __restrict__ mass) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  const double* fc = f + off[cell0 + b];
  double acc = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) acc += fc[r];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double ms = hd * red[0];
  if (threadIdx.x == 0) mass[b] = ms;
  const double inv = ms > 0.0 ? kInputScale / ms : 0.0;
  for (int r = threadIdx.x; r < n; r += 256) Fin[(int64_t)b * n + r] = (float)(fc[r] * inv);
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
template <int N, int K, int C>
struct FnoOps {
  using D = FnoDims<N, K>;
  static hipError_t fwd_transform(const float* u, int nsc, cx<float>* T, cx<float>* Uh,
                                  hipStream_t st) {
    hipLaunchKernelGGL((k_fno_fwd_slab<N, K>), dim3(nsc * N), dim3(N), 0, st, u, T);
    const int64_t nt = (int64_t)nsc * D::PEN;
    hipLaunchKernelGGL((k_fno_fwd_x<N, K, C>), dim3((unsigned)((nt + 63) / 64)), dim3(64), 0, st,
                       T, nsc, Uh);
    return hipGetLastError();
  }
  static hipError_t inv_transform(const cx<float>* V, int nsc, cx<float>* T, float* out,
                                  int accumulate, hipStream_t st) {
    const int64_t nt = (int64_t)nsc * D::PEN;
    hipLaunchKernelGGL((k_fno_inv_x<N, K, C>), dim3((unsigned)((nt + 63) / 64)), dim3(64), 0, st,
                       V, nsc, T);
    hipLaunchKernelGGL((k_fno_inv_slab<N, K>), dim3(nsc * N), dim3(N), 0, st, T, out, accumulate);
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
  hipLaunchKernelGGL((k_fno_lift<C>), dim3(gb), dim3(256), 0, st, a.Fin, B, n, a.Wl, a.bl, a.u[0]);
  for (int l = 0; l < a.L; ++l) {
    hipError_t e = O::fwd_transform(a.u[l], B * C, a.T, a.Uh[l], st);
    if (e != hipSuccess) return e;
    const int64_t nbmc = (int64_t)B * D::NM * C;
    hipLaunchKernelGGL((k_fno_mix2<C>), dim3((unsigned)((nbmc + 255) / 256)), dim3(256), 0, st,
                       a.R[l], a.Uh[l], B, D::NM, 0, 1.f / (float)n, a.V);
    e = O::inv_transform(a.V, B * C, a.T, a.s, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fno_pointwise<C>), dim3(gb), dim3(256), 0, st, a.u[l], a.s, B, n,
                       a.W[l], a.bias[l], l + 1 < a.L ? 1 : 0, a.h[l], a.u[l + 1]);
  }
  hipLaunchKernelGGL((k_fno_proj<C>), dim3(gb), dim3(256), 0, st, a.u[a.L], B, n, a.Wp, a.bp, a.y);
  return hipGetLastError();
}

template <int C>
static hipError_t dense_grad(int mode, const float* act, const float* g, int B, int n, float* part,
                             int part_blocks, float* out, hipStream_t st) {
  const int64_t total = (int64_t)B * n;
  const int npb = (int)((total + part_blocks - 1) / part_blocks);
  hipLaunchKernelGGL((k_fno_dense_partial<C>), dim3(part_blocks), dim3(256), 0, st, mode, act, g,
                     B, n, npb, part);
  const int nvals = mode == 0 ? C * C + C : (mode == 1 ? 2 * C : C + 1);
  hipLaunchKernelGGL((k_fno_dense_final<C>), dim3((nvals + 255) / 256), dim3(256), 0, st, part,
                     part_blocks, nvals, out);
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
  hipLaunchKernelGGL(k_fno_loss, dim3(B), dim3(256), 0, st, a.y, a.target, B, n, a.dy, a.loss_b);
  e = dense_grad<C>(2, a.u[a.L], a.dy, B, n, a.part, a.part_blocks, a.gWp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fno_proj_bwd<C>), dim3(gb), dim3(256), 0, st, a.dy, B, n, a.Wp, a.du);
  for (int l = a.L - 1; l >= 0; --l) {
    // dh (into a.dh), pointwise part of du_in (into a.du2)
    hipLaunchKernelGGL((k_fno_pointwise_bwd<C>), dim3(gb), dim3(256), 0, st, a.du, a.h[l], B, n,
                       a.W[l], l + 1 < a.L ? 1 : 0, a.dh, a.du2);
    e = dense_grad<C>(0, a.u[l], a.dh, B, n, a.part, a.part_blocks, a.gW[l], st);
    if (e != hipSuccess) return e;
    // spectral part: Gv = truncated DFT(dh); dR = sum_b Gv conj(Uh); Gu = conj(R)^T Gv
    e = O::fwd_transform(a.dh, B * C, a.T, a.V, st);
    if (e != hipSuccess) return e;
    const int64_t nmcc = (int64_t)D::NM * C * C;
    hipLaunchKernelGGL((k_fno_dR<C>), dim3((unsigned)((nmcc + 255) / 256)), dim3(256), 0, st, a.V,
                       a.Uh[l], B, D::NM, 1.f / (float)n, a.gR[l]);
    const int64_t nbmc = (int64_t)B * D::NM * C;
    hipLaunchKernelGGL((k_fno_mix2<C>), dim3((unsigned)((nbmc + 255) / 256)), dim3(256), 0, st,
                       a.R[l], a.V, B, D::NM, 1, 1.f / (float)n, a.V2);
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
                         int B, float* Fin, double* mass, hipStream_t st) {
  hipLaunchKernelGGL(k_fno_normalize, dim3(B), dim3(256), 0, st, f, off, cell0, n, hd, Fin, mass);
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

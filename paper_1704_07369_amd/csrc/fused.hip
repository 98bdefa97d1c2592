// Fused per-term kernel of the 3D operator for gfx950.
//
// The gain is sum_t Re c_t Im c_t with c_t = IDFT[gamma_t Fh] (section 4.1,
// eq. fastAlg; gamma_t = alpha_t + i beta_t carries N^-d, the weights and the
// filter), the loss l = Re IDFT[D Fh] (section 3.1.2).  A 3D FP64 volume of
// one term (N^3 complex, 512 KB at N = 32) does not fit in a CU's LDS, so the
// inverse transform along x is split by decimation in frequency with radix P:
// for the output rows x = P q + s,
//   c(Pq+s, y, z) = sum_{k'<N/P} e^{2 pi i k' q/(N/P)} G_s(k', y, z),
//   G_s(k', .) = e^{2 pi i k' s/N} sum_{j<P} e^{2 pi i j s/P} Zh(k' + jN/P, .),
// where Zh = gamma_t Fh is transformed along y and z first.  One workgroup
// owns one (cell, s): for every term it forms G_s straight from Fh and the
// term's table (the table read from L2, where every cell reuses it; Fh read
// once per workgroup for the planes kept in registers, from L2 per term for
// the rest, where the cell's P workgroups share it), runs the inverse transforms
// along z, y (register lines, LDS transposes) and x (length N/P), and adds
// Re c Im c into FP64 registers that cover its N^3/P output points.  The loss
// term goes first, so the accumulator starts at -F l.
//
// Block -> (cell, s): blocks b, b+8, ... land on one XCD, so the P workgroups
// of a cell share that XCD's L2 (cell = (b / 8P) * 8 + b % 8, s = (b / 8) % P).
// N = 16, 24 run k_fused (volume staged in LDS); N = 32 runs k_fused_col
// (volume in registers, exchanges through LDS and lane permutes).
#include "fused.h"

#include "fft.h"

// gather load groups the FP32 column kernel prefetches (col_prefetch)
#ifndef EFM_COL_PREFETCH
#define EFM_COL_PREFETCH 5
#endif

namespace efm {

// exp(2 pi i m / N) for a runtime m in [0, N): a select over the exact table
template <int N, typename R>
__device__ __forceinline__ cx<R> unit_root(int m) {
  cx<R> w = {(R)1, (R)0};
  if constexpr (N > 1) {
#pragma unroll
    for (int k = 1; k < N; ++k)
      if (m == k) w = {(R)Tw<N>::c[k], (R)Tw<N>::s[k]};
  }
  return w;
}

// forward DFT along x of every (cell, k2, k1) pencil of W[cell][x][k2][k1], in place
// (KZ = N / 2: the half-space layout W[cell][x][k2 < N/2][k1])
template <typename R, int N, int KZ = N>
__global__ __launch_bounds__(64) void k_fwdx(cx<R>* __restrict__ W, int ncells) {
  constexpr int P2 = KZ * N;
  const int64_t gid = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (gid >= (int64_t)ncells * P2) return;
  const int64_t cc = gid / P2;
  const int p = (int)(gid % P2);
  cx<R>* Wc = W + cc * N * P2 + p;
  cx<R> v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = Wc[(int64_t)k * P2];
  fft_line<N, -1>(v);
#pragma unroll
  for (int k = 0; k < N; ++k) Wc[(int64_t)k * P2] = v[k];
}

// The whole forward transform of one cell per workgroup (N = 16, 24, 32;
// N^2/2 threads), into the half-space layout W[cell][kx][k2 < N/2][k1]:
//  1. the cell is read in halves through LDS, so that consecutive lanes load
//     consecutive values; thread (xl, y), xl < N/2, then transforms the real
//     z lines of (xl, y) and (xl + N/2, y) as one complex line C = DFT(a + i b)
//     and separates the two half spectra, A(k) = (C(k) + conj C(-k)) / 2 and
//     B(k) = (C(k) - conj C(-k)) / 2i for k2 < N/2;
//  2. through LDS (real parts, then imaginary parts) thread (x, k2) collects
//     its y line and transforms it;
//  3. through LDS thread (k2, k1) collects its x line, transforms it and
//     stores the pencil (consecutive threads, consecutive k1).
// F is read once and W written once, half the device-memory bytes of a slab
// pass followed by an in-place x pass.  Rows of N + 1 elements keep the
// lanes of every LDS access on distinct banks.
template <typename R, int N>
__global__ __launch_bounds__(N * N / 2) void k_fwd3(const double* __restrict__ f,
                                                    const int64_t* __restrict__ off,
                                                    int64_t cell0, cx<R>* __restrict__ W) {
  constexpr int H = N / 2, LD = N + 1, S = H * LD, T = N * N / 2;
  __shared__ R lds[N * S];
  const int t = threadIdx.x;
  const int64_t cc = blockIdx.x;
  const int xl = t / N, y = t % N;          // stage 1
  const int x = t / H, k2 = t % H;          // stage 2
  cx<R> A[H], B[H];
  {
    // each half x < N/2, x >= N/2 of the cell (N^3/2 values, N per thread)
    // read with consecutive lanes on consecutive values, then its z lines
    // taken from LDS (line xl N + y of the half = row t)
    const double* fc = f + off[cell0 + cc];
    cx<R> v[N];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h) __syncthreads();
#pragma unroll
      for (int i = 0; i < N; ++i)             // value t + i N^2/2 of the half: (row xl + i H, z = y)
        lds[(xl + i * H) * LD + y] = (R)fc[(int64_t)h * H * N * N + t + i * T];
      __syncthreads();
#pragma unroll
      for (int z = 0; z < N; ++z) {
        if (h == 0) v[z].x = lds[t * LD + z];
        else v[z].y = lds[t * LD + z];
      }
    }
    __syncthreads();                        // the rows are read before the exchanges
    fft_line<N, -1>(v);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const cx<R> p = v[k], m = v[(N - k) % N];
      A[k] = {(R)0.5 * (p.x + m.x), (R)0.5 * (p.y - m.y)};
      B[k] = {(R)0.5 * (p.y + m.y), (R)0.5 * (m.x - p.x)};
    }
  }
  cx<R> u[N];
#pragma unroll
  for (int k = 0; k < H; ++k) {
    lds[(xl * H + k) * LD + y] = A[k].x;
    lds[((xl + H) * H + k) * LD + y] = B[k].x;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) u[i].x = lds[t * LD + i];   // t * LD = (x H + k2) LD
  __syncthreads();
#pragma unroll
  for (int k = 0; k < H; ++k) {
    lds[(xl * H + k) * LD + y] = A[k].y;
    lds[((xl + H) * H + k) * LD + y] = B[k].y;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) u[i].y = lds[t * LD + i];
  fft_line<N, -1>(u);                       // (x, k1, k2)
  cx<R> w[N];
  const int q2 = t / N, q1 = t % N;         // stage 3
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < N; ++k1) lds[x * S + k2 * LD + k1] = u[k1].x;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) w[i].x = lds[i * S + q2 * LD + q1];
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < N; ++k1) lds[x * S + k2 * LD + k1] = u[k1].y;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) w[i].y = lds[i * S + q2 * LD + q1];
  fft_line<N, -1>(w);
  cx<R>* Wc = W + cc * N * H * N + t;       // t = k2 N + k1
#pragma unroll
  for (int kx = 0; kx < N; ++kx) Wc[(int64_t)kx * H * N] = w[kx];
}

// forward transform of the fused schedules: the spectrum in the half-space
// layout.  k_fwd3 for batches that give every CU a cell; smaller batches
// (one workgroup per cell would leave most CUs idle and the cell's load
// latency exposed) take the slab pass and the in-place x pass, spread over
// N^2/2 and N^2/128 blocks per cell.  Events 0 and 1 bracket the forward
// transform, event 2 follows at once (no 3D schedule has a separate x pass).
// (the smallest batch for k_fwd3, measured on MI355X: at N = 32 the two
// kernels take 14 against 23 us for 32 cells, 24 against 21 us for 64; at
// N = 24 14 against 15 us for 64 cells, 16 against 15 for 96; at N = 16
// k_fwd3 is faster from one cell on)
template <int N>
constexpr int fwd3_min_cells() { return N == 16 ? 1 : (N == 24 ? 96 : 64); }

template <typename R, int N>
static hipError_t launch_fwd_half(const ChunkArgs& a, hipStream_t st) {
  if (a.ev) (void)hipEventRecord(a.ev[0], st);
  if (a.ncells >= fwd3_min_cells<N>()) {
    hipLaunchKernelGGL((k_fwd3<R, N>), dim3((unsigned)a.ncells), dim3(N * N / 2), 0, st, a.f,
                       a.off, a.cell0, (cx<R>*)a.W);
  } else {
    hipError_t e = launch_fwd_half_slabs(a, st);
    if (e != hipSuccess) return e;
    constexpr int KZ = N / 2;
    const int64_t pencils = (int64_t)a.ncells * KZ * N;
    hipLaunchKernelGGL((k_fwdx<R, N, KZ>), dim3((unsigned)((pencils + 63) / 64)), dim3(64), 0,
                       st, (cx<R>*)a.W, a.ncells);
  }
  if (a.ev) (void)hipEventRecord(a.ev[1], st);
  if (a.ev) (void)hipEventRecord(a.ev[2], st);
  return hipGetLastError();
}

// Planes k2 < C of this thread's Fh inputs kept in registers across terms
// (measured on MI355X, 1024 cells: more planes spill or cost occupancy)
template <int N, int P, int B>
constexpr int fh_cache() {
  return N == 16 && P == 2 && B == 8 ? 8 : 4;
}

template <int N, int P>
constexpr int fused_threads() { return N / P * N; }

// v exp(2 pi i M / P) for a compile-time M (free for P = 2, 4)
template <int P, int M, typename R>
__device__ __forceinline__ cx<R> root_mul(cx<R> v) {
  if constexpr (M % P == 0) return v;
  else return twiddle<P, +1>(v, M % P);
}

// G_s over the volume of one term, staged in LDS at vol[k'][k2][k1] (tables
// are [k0][k2][k1]).  Only the half space k2 < N/2 is read: gamma = alpha +
// i beta is real-pair and even in k and Fh of real F is Hermitian, so with
// A = alpha Fh, B = beta Fh at the inputs k_j = (a + NP j, k2, bq),
//   sum_j r^j Zh(k_j)  = SA + i SB,          SA = sum_j r^j A_j, SB likewise,
//   sum_j r^-j Zh(-k_j) = conj(SA) + i conj(SB),
// where r = exp(2 pi i S / P).  The mirrored inputs -k_j are the inputs of
// G_s(am, N - k2, bm) in the order that gives roots conj(r^j) and twiddle
// conj(tw) (am = -a mod NP, bm = -bq mod N).  The plane k2 = N/2 vanishes
// (sigma(N/2) = 0).
// SA += sum_j r^j alpha_j Fh_j, SB += sum_j r^j beta_j Fh_j, r = exp(2 pi i S / P),
// over j = JJ .. P-1 (compile-time recursion, so every root is a constant)
template <int P, int S, int JJ = 0, typename R>
__device__ __forceinline__ void accum_roots(const cx<R> (&g)[P], const cx<R> (&fv)[P], cx<R>& SA,
                                            cx<R>& SB) {
  if constexpr (JJ < P) {
    const R al = g[JJ].x, be = g[JJ].y;
    SA = cadd(SA, root_mul<P, JJ * S>(cx<R>{al * fv[JJ].x, al * fv[JJ].y}));
    SB = cadd(SB, root_mul<P, JJ * S>(cx<R>{be * fv[JJ].x, be * fv[JJ].y}));
    accum_roots<P, S, JJ + 1>(g, fv, SA, SB);
  }
}

// Raw buffer loads for the gather: the thread's byte offset sits in one
// register for the whole kernel and each load's constant plane offset in a
// scalar register, so no per-load address arithmetic reaches the vector ALU
// (64-bit address forms cost about three vector instructions per load).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <typename R>
__device__ __forceinline__ cx<R> buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  cx<R> o;
  if constexpr (sizeof(R) == 8) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    __builtin_memcpy(&o, &v, sizeof(o));
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    __builtin_memcpy(&o, &v, sizeof(o));
  }
  return o;
}

// one plane pair of G_s: the entry at (a, kk, bq) and its mirror
template <typename R, int N, int P, int S>
__device__ __forceinline__ void gather_store(const cx<R> (&g)[P], const cx<R> (&fv)[P], int kk,
                                             int a, int bq, int am, int bm, cx<R> tw,
                                             cx<R> twc, cx<R>* vol) {
  constexpr int LD = N + 1;
  cx<R> SA = {(R)0, (R)0}, SB = {(R)0, (R)0};
  accum_roots<P, S>(g, fv, SA, SB);
  const cx<R> zp = {SA.x - SB.y, SA.y + SB.x}, zm = {SA.x + SB.y, SB.x - SA.y};
  // s = 0: the twiddle is exp(0) = 1
  vol[(a * N + kk) * LD + bq] = S == 0 ? zp : cmul(tw, zp);
  if (kk > 0) vol[(am * N + (N - kk)) * LD + bm] = S == 0 ? zm : cmul(twc, zm);
}

template <typename R, int N, int P, int C, int S>
__device__ __forceinline__ void gather_term(const cx<R>* __restrict__ Gt,
                                            const cx<R>* __restrict__ Fc,
                                            const cx<R> (&fh)[C > 0 ? C : 1][P], int a, int bq,
                                            int am, int bm, cx<R> tw, cx<R>* vol) {
  constexpr int NP = N / P, LD = N + 1;
  constexpr unsigned E = sizeof(cx<R>), n = N * N * N;
  // planes per group: a group's loads are in flight together
  constexpr int GP = 4;
  static_assert((N / 2) % GP == 0 && C % GP == 0, "half-space planes come in whole groups");
  const cx<R> twc = {tw.x, -tw.y};
  // table entry ((a + NP j) N + k2) N + bq, spectrum ((a + NP j) N/2 + k2) N + bq
  const __amdgpu_buffer_rsrc_t gt = buf_rsrc(Gt, n * E), fr = buf_rsrc(Fc, n / 2 * E);
  const unsigned gvo = (unsigned)(a * N * N + bq) * E, fvo = (unsigned)(a * (N / 2) * N + bq) * E;
  // planes k2 < C: Fh from registers (compile-time indices), table from L2
#pragma unroll
  for (int k2 = 0; k2 < C; k2 += GP) {
    cx<R> gl[GP][P];
#pragma unroll
    for (int u = 0; u < GP; ++u) {
#pragma unroll
      for (int j = 0; j < P; ++j)
        gl[u][j] = buf_load<R>(gt, gvo, (unsigned)((NP * j * N + k2 + u) * N) * E);
    }
#pragma unroll
    for (int u = 0; u < GP; ++u)
      gather_store<R, N, P, S>(gl[u], fh[k2 + u], k2 + u, a, bq, am, bm, tw, twc, vol);
    __builtin_amdgcn_sched_barrier(0);  // keep the next group's loads behind this group
  }
  // remaining planes: both from L2
#pragma unroll 1
  for (int k2 = C; k2 < N / 2; k2 += GP) {
    cx<R> gl[GP][P], fl[GP][P];
#pragma unroll
    for (int u = 0; u < GP; ++u) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        gl[u][j] = buf_load<R>(gt, gvo, (unsigned)((NP * j * N + k2 + u) * N) * E);
        fl[u][j] = buf_load<R>(fr, fvo, (unsigned)((NP * j * (N / 2) + k2 + u) * N) * E);
      }
    }
#pragma unroll
    for (int u = 0; u < GP; ++u)
      gather_store<R, N, P, S>(gl[u], fl[u], k2 + u, a, bq, am, bm, tw, twc, vol);
  }
  vol[(a * N + N / 2) * LD + bq] = {(R)0, (R)0};
}

template <typename R, int N, int P, int C, int S = 0>
__device__ __forceinline__ void gather_term_s(int s, const cx<R>* __restrict__ Gt,
                                              const cx<R>* __restrict__ Fc,
                                              const cx<R> (&fh)[C > 0 ? C : 1][P], int a,
                                              int bq, int am, int bm, cx<R> tw, cx<R>* vol) {
  if (s == S) gather_term<R, N, P, C, S>(Gt, Fc, fh, a, bq, am, bm, tw, vol);
  else if constexpr (S + 1 < P)
    gather_term_s<R, N, P, C, S + 1>(s, Gt, Fc, fh, a, bq, am, bm, tw, vol);
}

// One term: gather G_s into vol, inverse passes along z and y (register
// lines, LDS transposes), then along x for each of the thread's P lines.
// LOSS (the first term, table D): acc = -F l; otherwise acc += Re c Im c.
template <typename R, int N, int P, int C, bool LOSS>
__device__ __forceinline__ void run_term(int s, const cx<R>* __restrict__ Gt,
                                         const cx<R>* __restrict__ Fc,
                                         const cx<R> (&fh)[C > 0 ? C : 1][P],
                                         int a, int bq, int am, int bm, cx<R> tw, cx<R>* vol,
                                         const double* __restrict__ fc, double (&acc)[P][N / P]) {
  constexpr int NP = N / P, T = NP * N, LD = N + 1;
  const int th = threadIdx.x;
  __syncthreads();                      // the previous term's x pass is done with vol
  gather_term_s<R, N, P, C>(s, Gt, Fc, fh, a, bq, am, bm, tw, vol);
  __syncthreads();                      // mirrored entries land in other threads' columns
  cx<R> v[N];
#pragma unroll
  for (int k2 = 0; k2 < N; ++k2) v[k2] = vol[(a * N + k2) * LD + bq];
  fft_line<N, +1>(v);                   // along z: (k', k1 = bq, z), same column
#pragma unroll
  for (int z = 0; z < N; ++z) vol[(a * N + z) * LD + bq] = v[z];
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < N; ++k1) v[k1] = vol[(a * N + bq) * LD + k1];
  fft_line<N, +1>(v);                   // along y: (k', y, z = bq)
  __syncthreads();
#pragma unroll
  for (int y = 0; y < N; ++y) vol[(a * N + y) * LD + bq] = v[y];
  __syncthreads();
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;        // (y, z) of this x line
    const int y = line / N, z = line % N;
    cx<R> u[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) u[q] = vol[(q * N + y) * LD + z];
    fft_line<NP, +1>(u);                // x = P q + s
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if constexpr (LOSS) acc[p][q] = -fc[((P * q + s) * N + y) * N + z] * (double)u[q].x;
      else acc[p][q] += (double)u[q].x * (double)u[q].y;
    }
  }
}

template <typename R, int N, int P>
__global__ __launch_bounds__(N / P * N) void k_fused(
    const cx<R>* __restrict__ Fh, const cx<R>* __restrict__ G, int J,
    const double* f, const int64_t* __restrict__ off, int64_t cell0, int ncells,
    double* Q, double dt) {
  constexpr int NP = N / P;             // x rows per workgroup
  constexpr int T = NP * N;             // threads
  constexpr int LD = N + 1;             // padded LDS row
  constexpr int n = N * N * N;
  __shared__ cx<R> vol[NP * N * LD];
  const int blk = blockIdx.x;
  const int s = (blk / 8) % P;
  const int cc = (blk / (8 * P)) * 8 + blk % 8;
  if (cc >= ncells) return;             // whole workgroup
  const int th = threadIdx.x;
  const int a = th / N;                 // k' (z and y passes)
  const int bq = th % N;                // k1 (z pass), z (y pass)
  const cx<R> tw = unit_root<N, R>((a * s) % N);
  const int am = (NP - a) % NP, bm = (N - bq) % N;   // mirror of (a, bq)

  const cx<R>* Fc = Fh + (int64_t)cc * (n / 2);   // half-space spectrum [k0][k2 < N/2][k1]
  const int64_t base = off[cell0 + cc];
  const double* fc = f + base;
  // this thread's half-space inputs of Fh (the first C planes), the same for
  // every term: kept in registers, so a term's gather reads its table and
  // only the remaining planes of Fh
  constexpr int C = fh_cache<N, P, (int)sizeof(R)>();
  cx<R> fh[C > 0 ? C : 1][P];
#pragma unroll
  for (int k2 = 0; k2 < C; ++k2) {
#pragma unroll
    for (int j = 0; j < P; ++j) fh[k2][j] = Fc[((a + NP * j) * (N / 2) + k2) * N + bq];
  }
  double acc[P][NP];
  // the loss term (last table entry) first, outside the loop, so that the
  // addresses of F are not kept live across the gain terms
  run_term<R, N, P, C, true>(s, G + (int64_t)(J - 1) * n, Fc, fh, a, bq, am, bm, tw, vol, fc, acc);
  for (int term = 0; term < J - 1; ++term)
    run_term<R, N, P, C, false>(s, G + (int64_t)term * n, Fc, fh, a, bq, am, bm, tw, vol, fc, acc);
  double* qc = Q + base;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;
    const int y = line / N, z = line % N;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int idx = ((P * q + s) * N + y) * N + z;
      qc[idx] = dt == 0.0 ? acc[p][q] : fc[idx] + dt * acc[p][q];
    }
  }
}

// ---------------------------------------------------------------------------
// Column form for N = 32 (same mathematics as k_fused above).
//
// k_fused stages the whole (N/P) x N x N term volume in LDS, so at N = 32 one
// workgroup fills a CU (P = 4 in FP64) and the gather of a term cannot
// overlap the transform passes of another.  Here the volume lives in
// registers (one z column, then one y line per thread) and only exchanges go
// through memory:
//   - the mirrored half-space entries of the gather go to their owner by a
//     lane permute: the owner of plane am = -a mod N/P is placed in the same
//     wave (wave w holds planes w and N/P - w; wave 0 holds 0 and N/P/2), and
//     the column bm = -bq mod N in the same half-wave;
//   - the z -> y transpose stays inside a half-wave (one plane): real parts,
//     then imaginary parts, through that plane's LDS rows;
//   - the y -> x exchange crosses waves: real parts, then imaginary parts,
//     through an (N/P) x N x (N+1) LDS array of reals.
// Splitting the exchanges into real and imaginary halves keeps one line of
// registers live (at most 256 registers per thread, two waves per SIMD).  P = 2
// (512 threads, 132 KiB in FP64) halves the gathered bytes per cell against
// P = 4 (two workgroups of 66 KiB per CU, whose gathers and transform passes
// interleave).
// ---------------------------------------------------------------------------

// LDS row stride (in reals) of the column kernel's exchange buffer: even, so
// that the rows of the z -> y transpose are 16-byte aligned and read as
// 128-bit words (N + 1 rows were read as 64-bit words; measured at 32^3,
// 1024 cells: FP64 3.26 -> 3.20 ms per launch)
template <int N>
constexpr int col_ld() { return N + 2; }

// v as held by lane src4 / 4 of this wave (a lane permute; no LDS storage)
__device__ __forceinline__ double lane_read(double v, int src4) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_bpermute(src4, (int)(b & 0xffffffff));
  const int hi = __builtin_amdgcn_ds_bpermute(src4, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_read(float v, int src4) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src4, __float_as_int(v)));
}
template <typename R>
__device__ __forceinline__ cx<R> lane_read(cx<R> v, int src4) {
  return {lane_read(v.x, src4), lane_read(v.y, src4)};
}

// 0, opaque to the optimizer: offsets a loop-invariant pointer so that
// addresses formed from it are not hoisted (the pointer keeps its address space)
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+s"(z));
  return z;
}

// LDS writes of this wave visible to its other lanes (and earlier reads done)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Gather load groups of the next term issued during a term's x pass (see
// prefetch_table): FP32 at split 2 only, where the spectrum lives in
// registers and 36 registers are left (5 of the 8 groups: 254 registers, no
// spill; 6 spill).  1024 cells of 32^3, FP32 launch of 512 cells: 1.039 ms
// with none, 0.998 / 0.973 / 0.955 ms with 2 / 3 / 4 groups, 5 another 1.8 %
// faster than 4.  None where the column and the FP64 accumulators fill the
// register file.
template <typename R, int N, int P>
constexpr int col_prefetch();

// Planes of the thread's spectrum inputs that the column kernel keeps in
// registers for every term: all N/2 of them in FP32 at split 2 (64 more
// registers, 219 in all; the gather then reads only the term table: 1024
// cells of 32^3, 1.12 -> 1.055 ms per launch), none otherwise (no room next
// to the FP64 column).
template <typename R, int N, int P>
constexpr int fh_regs() { return sizeof(R) == 4 && P == 2 ? N / 2 : 0; }

template <typename R, int N, int P>
constexpr int col_prefetch() { return fh_regs<R, N, P>() > 0 ? EFM_COL_PREFETCH : 0; }

// Gather of one term into the thread's z column v[k2] (plane a, column bq;
// col = a N^2 + bq indexes its first table entry, fcol = a N^2 / 2 + bq its
// first input in the half-space spectrum [k0][k2 < N/2][k1], unless fh holds
// them): entries k2 < N/2 from its own loads, k2 > N/2 from the mirror
// partner, whose lane is partner4 / 4.  One group of GP planes of loads is in
// flight at a time: issuing the next group's loads before combining this one
// measured 3.5 % slower in FP64 and no faster in FP32 -- the gather is bound
// by the bytes delivered into the CU, not by the round trip.
// one group of GP planes: table entries (a + NP j, k2 + u, bq) of the term
// (resource gt, thread offset gvo = col * sizeof(cx)) and spectrum entries of
// the half-space layout (resource fr, offset fvo = fcol * sizeof(cx))
template <typename R, int N, int P, int GP>
__device__ __forceinline__ void gather_load(__amdgpu_buffer_rsrc_t gt, __amdgpu_buffer_rsrc_t fr,
                                            unsigned gvo, unsigned fvo, int k2,
                                            cx<R> (&gl)[GP][P], cx<R> (&fl)[GP][P]) {
  constexpr int NP = N / P;
  constexpr unsigned E = sizeof(cx<R>);
#pragma unroll
  for (int u = 0; u < GP; ++u) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      gl[u][j] = buf_load<R>(gt, gvo, (unsigned)((NP * j * N + k2 + u) * N) * E);
      fl[u][j] = buf_load<R>(fr, fvo, (unsigned)((NP * j * (N / 2) + k2 + u) * N) * E);
    }
  }
}

// planes per group of gather loads in the column kernels (4 spill in FP64)
constexpr int COL_GP = 2;

// Table loads of the first KP groups of a term's gather (spectrum held in
// registers, fh_regs > 0), issued before the term starts: the column kernel
// sends them out for the next term while it runs this term's x pass, when the
// column registers are free and the load path idle.
template <typename R, int N, int P, int KP>
__device__ __forceinline__ void prefetch_table(const cx<R>* __restrict__ Gt, int col,
                                               cx<R> (&pre)[KP > 0 ? KP : 1][COL_GP][P]) {
  if constexpr (KP > 0) {
    constexpr unsigned E = sizeof(cx<R>), n = N * N * N;
    const __amdgpu_buffer_rsrc_t gt = buf_rsrc(Gt, n * E);
    const unsigned gvo = (unsigned)col * E;
#pragma unroll
    for (int g = 0; g < KP; ++g)
#pragma unroll
      for (int u = 0; u < COL_GP; ++u)
#pragma unroll
        for (int j = 0; j < P; ++j)
          pre[g][u][j] =
              buf_load<R>(gt, gvo, (unsigned)(((N / P) * j * N + g * COL_GP + u) * N) * E);
  }
}

template <typename R, int N, int P, int S, int DEPTH, int KP>
__device__ __forceinline__ void gather_col(const cx<R>* __restrict__ Gt,
                                           const cx<R>* __restrict__ Fc, int col, int fcol,
                                           int partner4, cx<R> tw,
                                           const cx<R> (&fh)[fh_regs<R, N, P>() ? N / 2 : 1][P],
                                           const cx<R> (&pre)[KP > 0 ? KP : 1][COL_GP][P],
                                           cx<R> (&v)[N]) {
  constexpr int GP = COL_GP;
  constexpr int NG = N / 2 / GP;
  constexpr bool FH = fh_regs<R, N, P>() > 0;
  static_assert(KP == 0 || (FH && DEPTH == 1 && KP < NG), "prefetch: table-only gathers");
  constexpr unsigned E = sizeof(cx<R>), n = N * N * N;
  const cx<R> twc = {tw.x, -tw.y};
  const __amdgpu_buffer_rsrc_t gt = buf_rsrc(Gt, n * E), fr = buf_rsrc(Fc, n / 2 * E);
  const unsigned gvo = (unsigned)col * E, fvo = (unsigned)fcol * E;
  // DEPTH groups of loads in flight (ring of DEPTH buffers)
  cx<R> gl[DEPTH][GP][P], fl[DEPTH][GP][P];
  auto load = [&](int g) {
    const int b = g % DEPTH;
    if (g < KP) {
#pragma unroll
      for (int u = 0; u < GP; ++u)
#pragma unroll
        for (int j = 0; j < P; ++j) gl[b][u][j] = pre[g < KP ? g : 0][u][j];
    } else if constexpr (FH) {
#pragma unroll
      for (int u = 0; u < GP; ++u)
#pragma unroll
        for (int j = 0; j < P; ++j)
          gl[b][u][j] = buf_load<R>(gt, gvo, (unsigned)(((N / P) * j * N + g * GP + u) * N) * E);
    } else {
      gather_load<R, N, P, GP>(gt, fr, gvo, fvo, g * GP, gl[b], fl[b]);
    }
  };
#pragma unroll
  for (int g = 0; g < DEPTH - 1; ++g) load(g);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g + DEPTH - 1 < NG) load(g + DEPTH - 1);
    __builtin_amdgcn_sched_barrier(0);  // this group's loads go out before its math
    const int b = g % DEPTH;
#pragma unroll
    for (int u = 0; u < GP; ++u) {
      const int kk = g * GP + u;
      cx<R> SA = {(R)0, (R)0}, SB = {(R)0, (R)0};
      if constexpr (FH) accum_roots<P, S>(gl[b][u], fh[kk], SA, SB);
      else accum_roots<P, S>(gl[b][u], fl[b][u], SA, SB);
      const cx<R> zp = {SA.x - SB.y, SA.y + SB.x}, zm = {SA.x + SB.y, SB.x - SA.y};
      // s = 0: the twiddle is exp(0) = 1
      v[kk] = S == 0 ? zp : cmul(tw, zp);
      if (kk > 0) v[N - kk] = lane_read(S == 0 ? zm : cmul(twc, zm), partner4);
    }
    __builtin_amdgcn_sched_barrier(0);  // and the next group's loads stay behind it
  }
  v[N / 2] = {(R)0, (R)0};
}

template <typename R, int N, int P, int DEPTH, int KP, int S = 0>
__device__ __forceinline__ void gather_col_s(int s, const cx<R>* __restrict__ Gt,
                                             const cx<R>* __restrict__ Fc, int col, int fcol,
                                             int partner4, cx<R> tw,
                                             const cx<R> (&fh)[fh_regs<R, N, P>() ? N / 2 : 1][P],
                                             const cx<R> (&pre)[KP > 0 ? KP : 1][COL_GP][P],
                                             cx<R> (&v)[N]) {
  if (s == S) gather_col<R, N, P, S, DEPTH, KP>(Gt, Fc, col, fcol, partner4, tw, fh, pre, v);
  else if constexpr (S + 1 < P)
    gather_col_s<R, N, P, DEPTH, KP, S + 1>(s, Gt, Fc, col, fcol, partner4, tw, fh, pre, v);
}

// The thread's spectrum inputs of the planes kept in registers (fh_regs)
template <typename R, int N, int P>
__device__ __forceinline__ void load_fh(const cx<R>* __restrict__ Fc, int fcol,
                                        cx<R> (&fh)[fh_regs<R, N, P>() ? N / 2 : 1][P]) {
  if constexpr (fh_regs<R, N, P>() > 0) {
#pragma unroll
    for (int k2 = 0; k2 < N / 2; ++k2)
#pragma unroll
      for (int j = 0; j < P; ++j) fh[k2][j] = Fc[fcol + ((N / P) * j * (N / 2) + k2) * N];
  }
}

template <typename R, int N, int P, bool LOSS, int DEPTH = 1, int KP = 0>
__device__ __forceinline__ void run_term_col(int s, const cx<R>* __restrict__ Gt,
                                             const cx<R>* __restrict__ Fc, int a, int bq,
                                             int partner4, cx<R> tw,
                                             const cx<R> (&fh)[fh_regs<R, N, P>() ? N / 2 : 1][P],
                                             R* buf, const double* __restrict__ fc,
                                             double (&acc)[P][N / P],
                                             cx<R> (&pre)[KP > 0 ? KP : 1][COL_GP][P],
                                             const cx<R>* __restrict__ Gnext) {
  constexpr int NP = N / P, T = NP * N, LD = col_ld<N>();
  const int th = threadIdx.x;
  // offset by an opaque zero, the addresses of F are formed here instead of
  // being hoisted out of the term loop
  const int z0 = opaque_zero();
  const double* fp = fc + z0;
  cx<R> v[N];
  gather_col_s<R, N, P, DEPTH, KP>(s, Gt, Fc, a * N * N + bq, a * N * N / 2 + bq, partner4, tw,
                                   fh, pre, v);
  fft_line<N, +1>(v);                   // along z: (k', k1 = bq, z)
  R* pl = buf + a * N * LD;             // this half-wave's plane
  __syncthreads();                      // every wave is done reading the previous term
  // z -> y transpose inside the half-wave, real parts then imaginary parts
#pragma unroll
  for (int z = 0; z < N; ++z) pl[z * LD + bq] = v[z].x;
  wave_sync();
#pragma unroll
  for (int k1 = 0; k1 < N; ++k1) v[k1].x = pl[bq * LD + k1];   // now the y line's
  wave_sync();
  // the imaginary parts are still those of the z column
#pragma unroll
  for (int z = 0; z < N; ++z) pl[z * LD + bq] = v[z].y;
  wave_sync();
#pragma unroll
  for (int k1 = 0; k1 < N; ++k1) v[k1].y = pl[bq * LD + k1];
  fft_line<N, +1>(v);                   // along y: (k', y, z = bq)
  wave_sync();
  // y -> x exchange across waves
#pragma unroll
  for (int y = 0; y < N; ++y) pl[y * LD + bq] = v[y].x;
  // unconditional (the caller passes a valid table after the last term too):
  // a branch here would split the block and change which products the
  // compiler contracts into FMAs, and FP32 results would no longer equal the
  // term-parallel kernel's bit for bit
  prefetch_table<R, N, P, KP>(Gnext, a * N * N + bq, pre);
  __syncthreads();
  cx<R> u[P][NP];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;        // (y, z) of this x line
    const int y = line / N, z = line % N;
#pragma unroll
    for (int q = 0; q < NP; ++q) u[p][q].x = buf[(q * N + y) * LD + z];
  }
  __syncthreads();
#pragma unroll
  for (int y = 0; y < N; ++y) pl[y * LD + bq] = v[y].y;
  __syncthreads();
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;
    const int y = line / N, z = line % N;
#pragma unroll
    for (int q = 0; q < NP; ++q) u[p][q].y = buf[(q * N + y) * LD + z];
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;
    const int y = line / N, z = line % N;
    fft_line<NP, +1>(u[p]);             // x = P q + s
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      if constexpr (LOSS) acc[p][q] = -fp[((P * q + s) * N + y) * N + z] * (double)u[p][q].x;
      else acc[p][q] += (double)u[p][q].x * (double)u[p][q].y;
    }
  }
}

template <typename R, int N, int P>
__global__ __launch_bounds__(N / P * N) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_fused_col(const cx<R>* __restrict__ Fh, const cx<R>* __restrict__ G, int J,
                 const double* f, const int64_t* __restrict__ off, int64_t cell0, int ncells,
                 double* Q, double dt) {
  static_assert(N == 32, "one half-wave per (plane, column) line");
  constexpr int NP = N / P, T = NP * N, LD = col_ld<N>(), n = N * N * N;
  static_assert(T % 64 == 0 && T / 64 == NP / 2, "two planes per wave");
  __shared__ R buf[NP * N * LD];
  const int blk = blockIdx.x;
  const int s = (blk / 8) % P;
  const int cc = (blk / (8 * P)) * 8 + blk % 8;
  if (cc >= ncells) return;             // whole workgroup
  const int th = threadIdx.x;
  const int w = th / 64, h = (th / 32) % 2, bq = th % 32;
  const int a = h == 0 ? w : (w == 0 ? NP / 2 : NP - w);
  const int bm = (N - bq) % N;
  // mirror partner (plane -a mod NP, column bm): other half-wave, except in
  // wave 0 whose planes 0 and NP/2 are their own mirrors
  const int partner4 = 4 * ((w == 0 ? h : 1 - h) * 32 + bm);
  const cx<R> tw = unit_root<N, R>((a * s) % N);
  const cx<R>* Fc = Fh + (int64_t)cc * (n / 2);   // half-space spectrum
  const int64_t base = off[cell0 + cc];
  const double* fc = f + base;
  double acc[P][NP];
  cx<R> fh[fh_regs<R, N, P>() ? N / 2 : 1][P];
  load_fh<R, N, P>(Fc, a * N * N / 2 + bq, fh);
  constexpr int KP = col_prefetch<R, N, P>();
  cx<R> pre[KP > 0 ? KP : 1][COL_GP][P];
  prefetch_table<R, N, P, KP>(G + (int64_t)(J - 1) * n, a * N * N + bq, pre);
  // the next term's table (after the last term: the first table again, a
  // valid address whose loads are not used)
  run_term_col<R, N, P, true, 1, KP>(s, G + (int64_t)(J - 1) * n, Fc, a, bq, partner4, tw, fh,
                                     buf, fc, acc, pre, G);
  for (int term = 0; term < J - 1; ++term)
    run_term_col<R, N, P, false, 1, KP>(s, G + (int64_t)term * n, Fc, a, bq, partner4, tw, fh,
                                        buf, fc, acc, pre,
                                        G + (int64_t)(term + 1 < J - 1 ? term + 1 : 0) * n);
  // fresh copies again, so that the output addresses are not shared with
  // (and kept live from) the loss term's reads of F
  const int z0 = opaque_zero();
  double* qc = Q + base + z0;
  const double* fe = fc + z0;
  const int se = s + z0;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;
    const int y = line / N, z = line % N;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int idx = ((P * q + se) * N + y) * N + z;
      qc[idx] = dt == 0.0 ? acc[p][q] : fe[idx] + dt * acc[p][q];
    }
  }
}

// Load groups of the gather in flight in the term-parallel kernel: with one
// workgroup per (cell, term, residue class) the load latency is exposed (one
// wave per SIMD), so the next group is issued before the current one is
// combined.  The fused kernel keeps one group: there two waves per SIMD and
// the gather's bandwidth bound leave nothing to hide.
constexpr int TERMS_DEPTH = 2;

// Term-parallel form of the column kernel for small batches: one workgroup
// per (cell, term, x residue s) runs that single term (the same run_term_col)
// and writes its products, or for the loss term -F l, to part[cell][term][n];
// k_terms_reduce then sums them per point in the fused kernel's order (loss,
// then the terms in order).  A batch of a few cells fills J P workgroups per
// cell instead of P, so the latency is about that of one term.
template <typename R, int N, int P>
__global__ __launch_bounds__(N / P * N) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_terms_col(const cx<R>* __restrict__ Fh, const cx<R>* __restrict__ G, int J,
                 const double* f, const int64_t* __restrict__ off, int64_t cell0, int ncells,
                 double* __restrict__ part) {
  static_assert(N == 32, "one half-wave per (plane, column) line");
  constexpr int NP = N / P, T = NP * N, LD = col_ld<N>(), n = N * N * N;
  __shared__ R buf[NP * N * LD];
  const int blk = blockIdx.x;
  const int s = (blk / 8) % P;
  const int cc = (blk / (8 * P)) * 8 + blk % 8;
  if (cc >= ncells) return;             // whole workgroup
  const int term = blockIdx.y;
  const int th = threadIdx.x;
  const int w = th / 64, h = (th / 32) % 2, bq = th % 32;
  const int a = h == 0 ? w : (w == 0 ? NP / 2 : NP - w);
  const int bm = (N - bq) % N;
  const int partner4 = 4 * ((w == 0 ? h : 1 - h) * 32 + bm);
  const cx<R> tw = unit_root<N, R>((a * s) % N);
  const cx<R>* Fc = Fh + (int64_t)cc * (n / 2);
  const double* fc = f + off[cell0 + cc];
  double acc[P][NP];
  cx<R> fh[fh_regs<R, N, P>() ? N / 2 : 1][P];
  load_fh<R, N, P>(Fc, a * N * N / 2 + bq, fh);
  cx<R> pre[1][COL_GP][P];                // no prefetch: one term per workgroup
  if (term == J - 1) {
    run_term_col<R, N, P, true, TERMS_DEPTH>(s, G + (int64_t)(J - 1) * n, Fc, a, bq, partner4,
                                             tw, fh, buf, fc, acc, pre, nullptr);
  } else {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int q = 0; q < NP; ++q) acc[p][q] = 0.0;
    run_term_col<R, N, P, false, TERMS_DEPTH>(s, G + (int64_t)term * n, Fc, a, bq, partner4,
                                              tw, fh, buf, fc, acc, pre, nullptr);
  }
  double* pc = part + ((int64_t)cc * J + term) * n;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;
    const int y = line / N, z = line % N;
#pragma unroll
    for (int q = 0; q < NP; ++q) pc[((P * q + s) * N + y) * N + z] = acc[p][q];
  }
}

// The same for the LDS-volume kernel (N = 16, 24): one workgroup per (cell,
// term, x residue class) runs that term with run_term and writes its products.
template <typename R, int N, int P>
__global__ __launch_bounds__(N / P * N) void k_terms_lds(
    const cx<R>* __restrict__ Fh, const cx<R>* __restrict__ G, int J, const double* f,
    const int64_t* __restrict__ off, int64_t cell0, int ncells, double* __restrict__ part) {
  constexpr int NP = N / P, T = NP * N, LD = N + 1, n = N * N * N;
  __shared__ cx<R> vol[NP * N * LD];
  const int blk = blockIdx.x;
  const int s = (blk / 8) % P;
  const int cc = (blk / (8 * P)) * 8 + blk % 8;
  if (cc >= ncells) return;             // whole workgroup
  const int term = blockIdx.y;
  const int th = threadIdx.x;
  const int a = th / N, bq = th % N;
  const cx<R> tw = unit_root<N, R>((a * s) % N);
  const int am = (NP - a) % NP, bm = (N - bq) % N;
  const cx<R>* Fc = Fh + (int64_t)cc * (n / 2);
  const double* fc = f + off[cell0 + cc];
  constexpr int C = fh_cache<N, P, (int)sizeof(R)>();
  cx<R> fh[C > 0 ? C : 1][P];
#pragma unroll
  for (int k2 = 0; k2 < C; ++k2) {
#pragma unroll
    for (int j = 0; j < P; ++j) fh[k2][j] = Fc[((a + NP * j) * (N / 2) + k2) * N + bq];
  }
  double acc[P][NP];
  if (term == J - 1) {
    run_term<R, N, P, C, true>(s, G + (int64_t)(J - 1) * n, Fc, fh, a, bq, am, bm, tw, vol, fc,
                               acc);
  } else {
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int q = 0; q < NP; ++q) acc[p][q] = 0.0;
    run_term<R, N, P, C, false>(s, G + (int64_t)term * n, Fc, fh, a, bq, am, bm, tw, vol, fc,
                                acc);
  }
  double* pc = part + ((int64_t)cc * J + term) * n;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int line = th + T * p;
    const int y = line / N, z = line % N;
#pragma unroll
    for (int q = 0; q < NP; ++q) pc[((P * q + s) * N + y) * N + z] = acc[p][q];
  }
}

// Q = sum of the term partials in the fused kernel's order (the loss term's
// -F l first); Euler update when dt != 0
__global__ __launch_bounds__(256) void k_terms_reduce(const double* __restrict__ part, int J,
                                                      int n, const double* f,
                                                      const int64_t* __restrict__ off,
                                                      int64_t cell0, int ncells, double* Q,
                                                      double dt) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)ncells * n) return;
  const int64_t cc = gid / n, r = gid % n;
  const double* pc = part + cc * J * n + r;
  double acc = pc[(int64_t)(J - 1) * n];
  // loads of 8 terms in flight, added in term order
  int t = 0;
  for (; t + 8 <= J - 1; t += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = pc[(int64_t)(t + k) * n];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += v[k];
  }
  for (; t < J - 1; ++t) acc += pc[(int64_t)t * n];
  const int64_t o = off[cell0 + cc] + r;
  Q[o] = dt == 0.0 ? acc : f[o] + dt * acc;
}

template <typename R, int N, int P>
static hipError_t launch_terms_t(const ChunkArgs& a, hipStream_t st) {
  cx<R>* W = (cx<R>*)a.W;
  hipError_t e = launch_fwd_half<R, N>(a, st);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((a.ncells + 7) / 8 * 8 * P), (unsigned)a.J);
  if constexpr (N == 32)
    hipLaunchKernelGGL((k_terms_col<R, N, P>), grid, dim3(fused_threads<N, P>()), 0, st,
                       (const cx<R>*)W, (const cx<R>*)a.gamma, a.J, a.f, a.off, a.cell0,
                       a.ncells, (double*)a.Z);
  else
    hipLaunchKernelGGL((k_terms_lds<R, N, P>), grid, dim3(fused_threads<N, P>()), 0, st,
                       (const cx<R>*)W, (const cx<R>*)a.gamma, a.J, a.f, a.off, a.cell0,
                       a.ncells, (double*)a.Z);
  return launch_terms_reduce(a, N * N * N, st);
}

hipError_t launch_terms_reduce(const ChunkArgs& a, int n, hipStream_t st) {
  const int64_t pts = (int64_t)a.ncells * n;
  hipLaunchKernelGGL(k_terms_reduce, dim3((unsigned)((pts + 255) / 256)), dim3(256), 0, st,
                     (const double*)a.Z, a.J, n, a.f, a.off, a.cell0, a.ncells, a.Q, a.dt);
  if (a.ev) (void)hipEventRecord(a.ev[3], st);
  return hipGetLastError();
}

bool terms_supported(int N, int precision, int split) {
  // the splits of the fused schedule
  return fused_supported(N, precision, split);
}

hipError_t launch_terms(const ChunkArgs& a, int split, hipStream_t st) {
  if (a.ncells <= 0) return hipSuccess;
  if (a.d == 2) return launch_terms_2d(a, st);
  if (a.d != 3 || !terms_supported(a.N, a.precision, split) || !a.Z) return hipErrorInvalidValue;
  if (a.precision == 0) {
    if (a.N == 16) return split == 1 ? launch_terms_t<double, 16, 1>(a, st)
                                     : launch_terms_t<double, 16, 2>(a, st);
    if (a.N == 24) return split == 2 ? launch_terms_t<double, 24, 2>(a, st)
                                     : launch_terms_t<double, 24, 3>(a, st);
    return split == 2 ? launch_terms_t<double, 32, 2>(a, st) : launch_terms_t<double, 32, 4>(a, st);
  }
  if (a.N == 16) return split == 1 ? launch_terms_t<float, 16, 1>(a, st)
                                   : launch_terms_t<float, 16, 2>(a, st);
  if (a.N == 24) return split == 2 ? launch_terms_t<float, 24, 2>(a, st)
                                   : launch_terms_t<float, 24, 3>(a, st);
  return split == 2 ? launch_terms_t<float, 32, 2>(a, st) : launch_terms_t<float, 32, 4>(a, st);
}

// the forward transform, then the fused kernel (COL: the column form); both
// forms read only the half space k2 < N/2 of the spectrum
template <typename R, int N, int P, bool COL>
static hipError_t launch_fused_t(const ChunkArgs& a, hipStream_t st) {
  cx<R>* W = (cx<R>*)a.W;
  hipError_t e = launch_fwd_half<R, N>(a, st);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)((a.ncells + 7) / 8 * 8 * P)), block(fused_threads<N, P>());
  if constexpr (COL)
    hipLaunchKernelGGL((k_fused_col<R, N, P>), grid, block, 0, st, (const cx<R>*)W,
                       (const cx<R>*)a.gamma, a.J, a.f, a.off, a.cell0, a.ncells, a.Q, a.dt);
  else
    hipLaunchKernelGGL((k_fused<R, N, P>), grid, block, 0, st, (const cx<R>*)W,
                       (const cx<R>*)a.gamma, a.J, a.f, a.off, a.cell0, a.ncells, a.Q, a.dt);
  if (a.ev) (void)hipEventRecord(a.ev[3], st);
  return hipGetLastError();
}

int fused_default_split(int N, int precision) {
  if (precision == 2) return 0;         // split-BF16 keeps its MFMA x pass
  switch (N) {
    case 16: return 1;
    case 24: return 3;
    case 32: return 2;
    default: return 0;
  }
}

bool fused_supported(int N, int precision, int split) {
  if (precision == 2) return false;
  switch (N) {
    case 16: return split == 1 || split == 2;
    case 24: return split == 2 || split == 3;
    case 32: return split == 2 || split == 4;
    default: return false;
  }
}

hipError_t launch_fused(const ChunkArgs& a, int split, hipStream_t st) {
  if (a.ncells <= 0) return hipSuccess;
  if (a.d != 3 || !fused_supported(a.N, a.precision, split)) return hipErrorInvalidValue;
  if (a.precision == 0) {
    if (a.N == 16) return split == 1 ? launch_fused_t<double, 16, 1, false>(a, st)
                                     : launch_fused_t<double, 16, 2, false>(a, st);
    if (a.N == 24) return split == 2 ? launch_fused_t<double, 24, 2, false>(a, st)
                                     : launch_fused_t<double, 24, 3, false>(a, st);
    return split == 2 ? launch_fused_t<double, 32, 2, true>(a, st)
                      : launch_fused_t<double, 32, 4, true>(a, st);
  }
  if (a.N == 16) return split == 1 ? launch_fused_t<float, 16, 1, false>(a, st)
                                   : launch_fused_t<float, 16, 2, false>(a, st);
  if (a.N == 24) return split == 2 ? launch_fused_t<float, 24, 2, false>(a, st)
                                   : launch_fused_t<float, 24, 3, false>(a, st);
  return split == 2 ? launch_fused_t<float, 32, 2, true>(a, st)
                    : launch_fused_t<float, 32, 4, true>(a, st);
}

}  // namespace efm

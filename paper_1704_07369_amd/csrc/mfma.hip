// Split-BF16 MFMA variant of the x pass (the pencil kernel) for the
// reduced-precision path.  For every term j the inverse DFT along x of
// Y = gamma_j Fh is a true contraction
//     [Re Z; Im Z] = [[C, -S], [S, C]] [Re Y; Im Y],   C, S = cos, sin(2 pi x k/N)
// i.e. a (2N x 2N) real matrix times (2N x pencils).  It runs on
// v_mfma_f32_32x32x16_bf16 with each operand split as v = hi + lo
// (hi = bf16(v), lo = bf16(v - hi)) and three products hi*hi + hi*lo + lo*hi
// (N = 16, 32, 64)
// accumulated in FP32 (about 16 significant bits per operand).  The forward
// DFT along x (once per pencil), the y/z passes (k_fwd, k_slab) and the
// storage stay FP32; the sum over terms stays FP64 (k_slab).
//
// One wave handles 32 consecutive pencils of one cell: lane l works on pencil
// l % 32 and on half h = l / 32 of the K rows.  MFMA 32x32x16 operand layout
// (checked on the device): A lane l holds A[l%32][8h .. 8h+7] of the 32x16
// tile, B lane l holds B[8h .. 8h+7][l%32], D lane l holds
// D[8(i/4) + 4h + i%4][l%32], i = 0..15.
#include <hip/hip_runtime.h>

#include "fft.h"
#include "mfma.h"

namespace efm {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;

// exact sign flip of 8 bf16 values
__device__ __forceinline__ bf16x8 neg8(bf16x8 v) {
  struct U4 { unsigned u[4]; };
  U4 w = __builtin_bit_cast(U4, v);
#pragma unroll
  for (int i = 0; i < 4; ++i) w.u[i] ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, w);
}

// k0 of the m-th spectral value a lane of half h holds (m < N/2)
template <int N>
__device__ __forceinline__ int kset(int h, int m) {
  return (m / 8) * 16 + h * 8 + (m % 8);
}

template <int N>
__global__ __launch_bounds__(64) void k_pencil_bf16(const cx<float>* __restrict__ W,
                                                    const cx<float>* __restrict__ G, int J,
                                                    int ncells, cx<float>* __restrict__ Z) {
  static_assert(N == 16 || N == 32 || N == 64, "split-BF16 x pass: N = 16, 32 or 64");
  constexpr int P = N * N;
  constexpr int NT = 2 * N / 32;      // output row tiles (Re/Im blocks of 32 rows)
  constexpr int NQ = 2 * N / 16;      // K chunks of 16 rows
  constexpr int NH = N / 2;           // spectral values per lane
  // N = 64: the 128 x 128 matrix does not fit in registers; its C and S blocks
  // (hi, lo) live in LDS by (row tile, K chunk, lane) and the tiles of
  // [[C, -S], [S, C]] are assembled from them
  constexpr bool ALDS = N == 64;
  constexpr int AT = ALDS ? NT / 2 : 1, AQ = ALDS ? NQ / 2 : 1;
  __shared__ cx<float> fh[N][32];
  __shared__ bf16x8 cs_lds[ALDS ? 2 : 1][AT][AQ][2][64];   // [C, S][row tile][K chunk][hi, lo][lane]
  const int l = threadIdx.x, col = l % 32, h = l / 32;
  const int64_t pb = blockIdx.x;                    // block of 32 pencils
  const int cc = (int)(pb / (P / 32));
  const int p = (int)(pb % (P / 32)) * 32 + col;
  const bool active = cc < ncells;
  const int ccs = active ? cc : 0;

  // A operand: the real 2N x 2N inverse DFT matrix, split hi/lo
  constexpr int RR = ALDS ? 1 : NT, RQ = ALDS ? 1 : NQ;
  bf16x8 ahi[RR][RQ], alo[RR][RQ];
  if constexpr (!ALDS) {
#pragma unroll
    for (int R = 0; R < NT; ++R) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int r = R * 32 + col;                 // output row
          const int kr = q * 16 + h * 8 + j;          // K row
          const bool oim = r >= N, iim = kr >= N;
          const int x = oim ? r - N : r, k0 = iim ? kr - N : kr;
          double sn, cs;
          sincospi(2.0 * (double)((x * k0) % N) / (double)N, &sn, &cs);
          const double v = (!oim && !iim) ? cs : (!oim && iim) ? -sn : (oim && !iim) ? sn : cs;
          const __bf16 hi = (__bf16)(float)v;
          ahi[R][q][j] = hi;
          alo[R][q][j] = (__bf16)((float)v - (float)hi);
        }
      }
    }
  } else {
    for (int R = 0; R < AT; ++R) {
      for (int q = 0; q < AQ; ++q) {
        bf16x8 chi, clo, shi, slo;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int x = R * 32 + col, k0 = q * 16 + h * 8 + j;
          double sn, cs;
          sincospi(2.0 * (double)((x * k0) % N) / (double)N, &sn, &cs);
          const __bf16 ch = (__bf16)(float)cs, sh = (__bf16)(float)sn;
          chi[j] = ch;
          clo[j] = (__bf16)((float)cs - (float)ch);
          shi[j] = sh;
          slo[j] = (__bf16)((float)sn - (float)sh);
        }
        cs_lds[0][R][q][0][l] = chi;
        cs_lds[0][R][q][1][l] = clo;
        cs_lds[1][R][q][0][l] = shi;
        cs_lds[1][R][q][1][l] = slo;
      }
    }
  }

  // forward DFT along x of the 32 pencils (lanes of half 0), via LDS
  if (h == 0) {
    cx<float> v[N];
    const cx<float>* Wc = W + (int64_t)ccs * N * P + p;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = Wc[(int64_t)k * P];
    fft_line<N, -1>(v);
#pragma unroll
    for (int k = 0; k < N; ++k) fh[k][col] = v[k];
  }
  __syncthreads();
  cx<float> fl[NH];
#pragma unroll
  for (int m = 0; m < NH; ++m) fl[m] = fh[kset<N>(h, m)][col];

  for (int j = 0; j < J; ++j) {
    const cx<float>* Gj = G + (int64_t)j * N * P + p;
    float yre[NH], yim[NH];
#pragma unroll
    for (int m = 0; m < NH; ++m) {
      const cx<float> y = cmul(Gj[(int64_t)kset<N>(h, m) * P], fl[m]);
      yre[m] = y.x;
      yim[m] = y.y;
    }
    floatx16 acc[NT];
#pragma unroll
    for (int R = 0; R < NT; ++R)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[R][i] = 0.f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      bf16x8 bhi, blo;
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int m = (q % (NQ / 2)) * 8 + jj;      // Re rows first, then Im rows
        const float v = (q < NQ / 2) ? yre[m] : yim[m];
        const __bf16 hi = (__bf16)v;
        bhi[jj] = hi;
        blo[jj] = (__bf16)(v - (float)hi);
      }
#pragma unroll
      for (int R = 0; R < NT; ++R) {
        bf16x8 ah, al;
        if constexpr (ALDS) {
          // Re rows x Re cols: C; Re x Im: -S; Im x Re: S; Im x Im: C
          const bool re_out = R < NT / 2, re_in = q < NQ / 2;
          const int blk = re_out != re_in ? 1 : 0;
          ah = cs_lds[blk][R % AT][q % AQ][0][l];
          al = cs_lds[blk][R % AT][q % AQ][1][l];
          if (re_out && !re_in) {
            ah = neg8(ah);
            al = neg8(al);
          }
        } else {
          ah = ahi[R % RR][q % RQ];
          al = alo[R % RR][q % RQ];
        }
        acc[R] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bhi, acc[R], 0, 0, 0);
        acc[R] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, blo, acc[R], 0, 0, 0);
        acc[R] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bhi, acc[R], 0, 0, 0);
      }
    }
    if (active) {
      cx<float>* Zj = Z + ((int64_t)ccs * J + j) * N * P + p;
      if constexpr (N == 64) {
        // tiles 0, 1 rows = Re Z(x), x = 32 R + ..; tiles 2, 3 the matching Im Z(x)
#pragma unroll
        for (int R = 0; R < 2; ++R)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int x = 32 * R + 8 * (i / 4) + 4 * h + (i % 4);
            Zj[(int64_t)x * P] = {acc[R][i], acc[R + 2][i]};
          }
      } else if constexpr (N == 32) {
        // tile 0 rows = Re Z(x), tile 1 rows = Im Z(x), same x per (lane, i)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int x = 8 * (i / 4) + 4 * h + (i % 4);
          Zj[(int64_t)x * P] = {acc[0][i], acc[1][i]};
        }
      } else {
        // one tile: rows 0..15 = Re Z(x), rows 16..31 = Im Z(x)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int x = 8 * (i / 4) + 4 * h + (i % 4);
          Zj[(int64_t)x * P] = {acc[0][i], acc[0][i + 8]};
        }
      }
    }
  }
}

hipError_t launch_pencil_bf16(const void* W, const void* G, int J, int ncells, void* Z, int N,
                              hipStream_t st) {
  if (ncells <= 0) return hipSuccess;
  const int blocks = ncells * N * N / 32;
  if (N == 64) {
    hipLaunchKernelGGL(k_pencil_bf16<64>, dim3(blocks), dim3(64), 0, st, (const cx<float>*)W,
                       (const cx<float>*)G, J, ncells, (cx<float>*)Z);
  } else if (N == 32) {
    hipLaunchKernelGGL(k_pencil_bf16<32>, dim3(blocks), dim3(64), 0, st, (const cx<float>*)W,
                       (const cx<float>*)G, J, ncells, (cx<float>*)Z);
  } else if (N == 16) {
    hipLaunchKernelGGL(k_pencil_bf16<16>, dim3(blocks), dim3(64), 0, st, (const cx<float>*)W,
                       (const cx<float>*)G, J, ncells, (cx<float>*)Z);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace efm

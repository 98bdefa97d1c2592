// Launch interface of the Fourier-neural-operator surrogate kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.h"

namespace efm {

constexpr int FNO_MAX_LAYERS = 8;
// blocks per cell of the per-cell reductions (n is a multiple of it)
constexpr int RED_CHUNKS = 16;

// Device pointers of one forward/backward pass over B cells (all FP32 unless
// noted).  n = N^3, NM = 4 K^3 kept modes, C channels, L layers.
struct FnoArgs {
  int N = 0, K = 0, C = 0, L = 0, B = 0;
  bool store_h = true;                // keep the pre-activations (needed by the backward pass)
  // parameters
  const float* Wl = nullptr;          // [C]
  const float* bl = nullptr;          // [C]
  const float* W[FNO_MAX_LAYERS] = {};      // [C][C] (out, in)
  const float* bias[FNO_MAX_LAYERS] = {};   // [C]
  const cx<float>* R[FNO_MAX_LAYERS] = {};  // [NM][C][C] (mode, in, out)
  const float* Wp = nullptr;          // [C]
  const float* bp = nullptr;          // [1]
  // gradients (same layouts; gWl = [Wl, bl], gW[l] = [W, bias], gWp = [Wp, bp])
  float* gWl = nullptr;
  float* gW[FNO_MAX_LAYERS] = {};
  cx<float>* gR[FNO_MAX_LAYERS] = {};
  float* gWp = nullptr;
  // activations and scratch
  const float* Fin = nullptr;         // [B][n]  normalised input
  const float* target = nullptr;      // [B][n]  normalised target (training)
  float* u[FNO_MAX_LAYERS + 1] = {};  // [B][C][n]
  float* h[FNO_MAX_LAYERS] = {};      // [B][C][n] pre-activations
  cx<float>* Uh[FNO_MAX_LAYERS] = {}; // [B][NM][C] kept modes of u[l]
  cx<float>* T = nullptr;             // [B*C][N][2K*K] transform intermediate
  cx<float>* V = nullptr;             // [B][NM][C]
  cx<float>* V2 = nullptr;            // [B][NM][C]
  float* y = nullptr;                 // [B][n] prediction
  float* dy = nullptr;                // [B][n]
  float* du = nullptr;                // [B][C][n]
  float* du2 = nullptr;               // [B][C][n]
  float* dh = nullptr;                // [B][C][n]
  double* loss_b = nullptr;           // [B]
  float* part = nullptr;              // [part_blocks][C*C+C]
  int part_blocks = 0;
};

bool fno_supported(int N, int K, int C);
hipError_t fno_forward(const FnoArgs& a, hipStream_t st);
hipError_t fno_backward(const FnoArgs& a, hipStream_t st);   // needs a prior forward
hipError_t fno_adam(float* p, const float* g, float* m, float* v, int64_t np, float lr, float b1,
                    float b2, float eps, int step, hipStream_t st);
// part: RED_CHUNKS B doubles of scratch
hipError_t fno_normalize(const double* f, const int64_t* off, int64_t cell0, int n, double hd,
                         int B, double* part, float* Fin, double* mass, hipStream_t st);
hipError_t fno_target(const double* Q, const int64_t* off, int64_t cell0, int n, int B,
                      const double* mass, float* t, hipStream_t st);
hipError_t fno_denormalize(const float* y, const double* mass, const int64_t* off, int64_t cell0,
                           int n, int B, double* Q, hipStream_t st);

}  // namespace efm

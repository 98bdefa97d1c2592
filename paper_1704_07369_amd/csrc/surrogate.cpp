// Learned surrogate of the collision operator (C ABI part): a Fourier neural
// operator trained on (F, Q) pairs produced by the exact operator, screened by
// the discrete H-functional sign and moment residuals, with fallback to the
// exact operator for every cell that fails the screen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/ec.h"
#include "fno.h"
#include "internal.h"

using namespace efm;

namespace {

#define SCHK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return set_error(EC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename F>
int sguard(F&& fn) {
  try {
    return fn();
  } catch (const std::bad_alloc&) {
    return set_error(EC_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(EC_ERR_ARG, e.what());
  } catch (...) {
    return set_error(EC_ERR_ARG, "unknown exception");
  }
}

}  // namespace

struct ec_surrogate {
  int N = 0, K = 0, C = 0, L = 0, maxB = 0;
  int64_t n = 0, NM = 0, nparams = 0;
  // parameter block offsets (in floats)
  int64_t oWl = 0, obl = 0, oW[FNO_MAX_LAYERS] = {}, ob[FNO_MAX_LAYERS] = {},
          oR[FNO_MAX_LAYERS] = {}, oWp = 0, obp = 0;
  float* d_p = nullptr;   // parameters
  float* d_g = nullptr;   // gradients
  float* d_m = nullptr;   // Adam moments
  float* d_v = nullptr;
  int adam_step = 0;
  // activations
  std::vector<void*> bufs;
  FnoArgs a;
  float* d_Fin = nullptr;
  double* d_mass = nullptr;
  double* d_red = nullptr;      // [max_batch][RED_CHUNKS][6] partial sums of the reductions
  double* d_screen = nullptr;   // [cells][4]: P, mass, momentum, energy residual
  int32_t* d_flag = nullptr;
  double* d_fc = nullptr;       // compact fallback cells (owned batch layout)
  double* d_qc = nullptr;
  int64_t* d_idx = nullptr;
  int64_t scap = 0;             // capacity of d_flag / d_screen / d_idx (cells)
  ec_batch* fb = nullptr;       // fallback batch (capacity fb_cap cells)
  int64_t fb_cap = 0;
  const ec_plan* plan = nullptr;
};

namespace {

hipError_t dalloc(ec_surrogate* s, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) s->bufs.push_back(*p);
  return e;
}

// ---- screening kernels -------------------------------------------------------
// per cell: P = h^d sum_{F>0} Q ln F of the projected Q; the raw prediction's
// moment residuals were written to out[c*4 + 1..3] by the projection
__global__ __launch_bounds__(256) void k_screen(const double* __restrict__ f,
                                                const double* __restrict__ Q,
                                                const int64_t* __restrict__ off, int N, double L,
                                                double tau_m, double tau_e, double* __restrict__ out,
                                                int32_t* __restrict__ flag) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const double* fc = f + off[c];
  const double* qc = Q + off[c];
  const int n = N * N * N;
  const double h = 2.0 * L / N;
  double a = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) {
    const double fv = fc[r];
    if (fv > 0.0) a += qc[r] * log(fv);
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = out + (int64_t)c * 4;
    const double P = h * h * h * red[0];
    o[0] = P;
    const double mass_res = o[1], mom_res = o[2], en_res = o[3];
    // tau_m < 0: screen disabled, every cell keeps the prediction;
    // tau_e < 0: no momentum and energy checks (the exact operator conserves
    // neither exactly on the grid, and their residuals do not single out the
    // cells the network predicts worst)
    const bool moments_ok = tau_e < 0.0 || ((mom_res <= tau_e) && (en_res <= tau_e));
    const bool ok = tau_m < 0.0 ||
                    ((P <= 0.0) && (mass_res <= tau_m) && moments_ok && isfinite(P) &&
                     isfinite(mass_res));
    flag[c] = ok ? 0 : 1;
  }
}

// ---- mass projection -------------------------------------------------------
// Q <- Q - (sum_r Q) / n: the orthogonal (Euclidean) projection onto grid
// functions with zero discrete mass.  The exact operator conserves mass
// exactly (momentum and energy only to spectral accuracy), so this projection
// never moves the prediction farther from it in the 2-norm.  Before
// projecting, the raw prediction's residuals |sum Q| / sum|Q|,
// |sum Q v| / (L sum|Q|) and |sum Q |v|^2| / (3 L^2 sum|Q|) go to
// out[c*4 + 1..3] for the screen.  Grid (RED_CHUNKS, cells cell0 ..): the
// first kernel writes six partial sums per chunk, the second adds them in a
// fixed order and projects its chunk.
constexpr int NMOM = 6;

__global__ __launch_bounds__(256) void k_project_partial(const double* __restrict__ Q,
                                                         const int64_t* __restrict__ off,
                                                         int64_t cell0, int N, double L,
                                                         double* __restrict__ part) {
  __shared__ double red[NMOM][256];
  const int b = blockIdx.y, j = blockIdx.x;
  const int n = N * N * N, chunk = n / RED_CHUNKS;
  const double* qc = Q + off[cell0 + b];
  const double h = 2.0 * L / N;
  double a[NMOM] = {0, 0, 0, 0, 0, 0};
  for (int r = j * chunk + threadIdx.x; r < (j + 1) * chunk; r += 256) {
    const int ix = r / (N * N), iy = (r / N) % N, iz = r % N;
    const double vx = -L + ix * h, vy = -L + iy * h, vz = -L + iz * h;
    const double q = qc[r];
    a[0] += q;
    a[1] += q * vx;
    a[2] += q * vy;
    a[3] += q * vz;
    a[4] += q * (vx * vx + vy * vy + vz * vz);
    a[5] += fabs(q);
  }
#pragma unroll
  for (int k = 0; k < NMOM; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < NMOM; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < NMOM)
    part[((int64_t)b * RED_CHUNKS + j) * NMOM + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_project(double* __restrict__ Q,
                                                 const int64_t* __restrict__ off, int64_t cell0,
                                                 int N, double L, const double* __restrict__ part,
                                                 double* __restrict__ out) {
  const int b = blockIdx.y, j = blockIdx.x;
  const int n = N * N * N, chunk = n / RED_CHUNKS;
  double m[NMOM] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < RED_CHUNKS; ++k)
#pragma unroll
    for (int q = 0; q < NMOM; ++q) m[q] += part[((int64_t)b * RED_CHUNKS + k) * NMOM + q];
  const int64_t c = cell0 + b;
  if (j == 0 && threadIdx.x == 0) {
    const double sabs = m[5] > 0.0 ? m[5] : 1e-300;
    double* o = out + c * 4;
    o[1] = fabs(m[0]) / sabs;
    o[2] = sqrt(m[1] * m[1] + m[2] * m[2] + m[3] * m[3]) / (sabs * L);
    o[3] = fabs(m[4]) / (3.0 * L * L * sabs);
  }
  const double mean = m[0] / n;
  double* qc = Q + off[c];
  for (int r = j * chunk + threadIdx.x; r < (j + 1) * chunk; r += 256) qc[r] -= mean;
}

// gather cells idx[j] of (f, off) into the compact layout (cell j at j * n)
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ f,
                                                const int64_t* __restrict__ off,
                                                const int64_t* __restrict__ idx, int64_t k, int n,
                                                const int64_t* __restrict__ coff,
                                                double* __restrict__ fc) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= k * n) return;
  const int64_t j = gid / n, r = gid % n;
  fc[coff[j] + r] = f[off[idx[j]] + r];
}

__global__ __launch_bounds__(256) void k_scatter(const double* __restrict__ qc,
                                                 const int64_t* __restrict__ coff,
                                                 const int64_t* __restrict__ idx, int64_t k, int n,
                                                 const int64_t* __restrict__ off,
                                                 double* __restrict__ Q) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= k * n) return;
  const int64_t j = gid / n, r = gid % n;
  Q[off[idx[j]] + r] = qc[coff[j] + r];
}

void bind_params(ec_surrogate* s) {
  FnoArgs& a = s->a;
  a.Wl = s->d_p + s->oWl;
  a.bl = s->d_p + s->obl;
  a.gWl = s->d_g + s->oWl;
  for (int l = 0; l < s->L; ++l) {
    a.W[l] = s->d_p + s->oW[l];
    a.bias[l] = s->d_p + s->ob[l];
    a.R[l] = (const cx<float>*)(s->d_p + s->oR[l]);
    a.gW[l] = s->d_g + s->oW[l];
    a.gR[l] = (cx<float>*)(s->d_g + s->oR[l]);
  }
  a.Wp = s->d_p + s->oWp;
  a.bp = s->d_p + s->obp;
  a.gWp = s->d_g + s->oWp;
}

// forward of B cells of one batch (cells cell0 .. cell0+B-1) into Q, then the
// conservative projection
int forward_batch_cells(ec_surrogate* s, const ec_batch* batch, const double* f, double* Q,
                        int64_t cell0, int B, hipStream_t st) {
  const double L = plan_L(batch_group_plan(batch, 0));
  const double h = 2.0 * L / s->N;
  SCHK(fno_normalize(f, batch_offsets_dev(batch), cell0, (int)s->n, h * h * h, B, s->d_red,
                     s->d_Fin, s->d_mass, st));
  FnoArgs a = s->a;
  a.B = B;
  a.Fin = s->d_Fin;
  a.store_h = false;
  SCHK(fno_forward(a, st));
  SCHK(fno_denormalize(a.y, s->d_mass, batch_offsets_dev(batch), cell0, (int)s->n, B, Q, st));
  const dim3 grid(RED_CHUNKS, (unsigned)B);
  hipLaunchKernelGGL(k_project_partial, grid, dim3(256), 0, st, Q, batch_offsets_dev(batch), cell0,
                     s->N, L, s->d_red);
  hipLaunchKernelGGL(k_project, grid, dim3(256), 0, st, Q, batch_offsets_dev(batch), cell0, s->N, L,
                     s->d_red, s->d_screen);
  SCHK(hipGetLastError());
  return EC_OK;
}

}  // namespace

extern "C" {

int ec_surrogate_create(int N, int modes, int channels, int layers, uint64_t seed, int max_batch,
                        ec_surrogate** out) {
  return sguard([&]() -> int {
    if (!out) return set_error(EC_ERR_ARG, "out is null");
    *out = nullptr;
    if (!fno_supported(N, modes, channels))
      return set_error(EC_ERR_UNSUPPORTED,
                       "surrogate sizes: (N, modes, channels) = (32,12,16), (16,6,8) or (8,2,4)");
    if (layers < 1 || layers > FNO_MAX_LAYERS || max_batch < 1)
      return set_error(EC_ERR_ARG, "need 1 <= layers <= 8 and max_batch >= 1");
    auto* s = new ec_surrogate();
    s->N = N; s->K = modes; s->C = channels; s->L = layers; s->maxB = max_batch;
    s->n = (int64_t)N * N * N;
    s->NM = 4LL * modes * modes * modes;
    const int C = channels;
    int64_t o = 0;
    s->oWl = o; o += C;
    s->obl = o; o += C;
    for (int l = 0; l < layers; ++l) {
      s->oW[l] = o; o += (int64_t)C * C;
      s->ob[l] = o; o += C;
      s->oR[l] = o; o += 2 * s->NM * C * C;
    }
    s->oWp = o; o += C;
    s->obp = o; o += 1;
    s->nparams = o;
    // seeded initialisation (host): uniform(-a, a) per block
    std::vector<float> p(o, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int64_t off, int64_t cnt, double amp) {
      std::uniform_real_distribution<double> U(-amp, amp);
      for (int64_t i = 0; i < cnt; ++i) p[off + i] = (float)U(rng);
    };
    fill(s->oWl, C, 1.0);
    fill(s->obl, C, 0.1);
    for (int l = 0; l < layers; ++l) {
      fill(s->oW[l], (int64_t)C * C, 1.0 / std::sqrt((double)C));
      fill(s->ob[l], C, 0.0);
      // spectral weights (the 1/n of the inverse transform is applied in the mixing)
      fill(s->oR[l], 2 * s->NM * C * C, 1.0 / ((double)C * C));
    }
    fill(s->oWp, C, 1.0 / std::sqrt((double)C));
    fill(s->obp, 1, 0.0);

    const size_t P = (size_t)o * sizeof(float);
    const int B = max_batch;
    const size_t act = (size_t)B * C * s->n * sizeof(float);
    const size_t mod = (size_t)B * s->NM * C * sizeof(cx<float>);
    const size_t T = (size_t)B * C * N * (2 * modes * modes) * sizeof(cx<float>);
    void* ptr = nullptr;
    bool ok = true;
    auto A = [&](size_t bytes) -> void* {
      if (!ok) return nullptr;
      if (dalloc(s, &ptr, bytes) != hipSuccess) { ok = false; return nullptr; }
      return ptr;
    };
    s->d_p = (float*)A(P);
    s->d_g = (float*)A(P);
    s->d_m = (float*)A(P);
    s->d_v = (float*)A(P);
    FnoArgs& a = s->a;
    a.N = N; a.K = modes; a.C = C; a.L = layers; a.B = B;
    for (int l = 0; l <= layers; ++l) a.u[l] = (float*)A(act);
    for (int l = 0; l < layers; ++l) {
      a.h[l] = (float*)A(act);
      a.Uh[l] = (cx<float>*)A(mod);
    }
    a.T = (cx<float>*)A(T);
    a.V = (cx<float>*)A(mod);
    a.V2 = (cx<float>*)A(mod);
    a.y = (float*)A((size_t)B * s->n * sizeof(float));
    a.dy = (float*)A((size_t)B * s->n * sizeof(float));
    a.du = (float*)A(act);
    a.du2 = (float*)A(act);
    a.dh = (float*)A(act);
    a.loss_b = (double*)A((size_t)B * sizeof(double));
    a.part_blocks = 2048;
    a.part = (float*)A((size_t)a.part_blocks * (C * C + C) * sizeof(float));
    s->d_Fin = (float*)A((size_t)B * s->n * sizeof(float));
    s->d_mass = (double*)A((size_t)B * sizeof(double));
    s->d_red = (double*)A((size_t)B * RED_CHUNKS * NMOM * sizeof(double));
    if (!ok) { ec_surrogate_destroy(s); return set_error(EC_ERR_OOM, "surrogate buffers"); }
    bind_params(s);
    if (hipMemcpy(s->d_p, p.data(), P, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->d_g, 0, P) != hipSuccess || hipMemset(s->d_m, 0, P) != hipSuccess ||
        hipMemset(s->d_v, 0, P) != hipSuccess) {
      ec_surrogate_destroy(s);
      return set_error(EC_ERR_DEVICE, "surrogate initialisation");
    }
    *out = s;
    return EC_OK;
  });
}

int ec_surrogate_destroy(ec_surrogate* s) {
  if (!s) return EC_OK;
  if (s->fb) ec_batch_destroy(s->fb);
  if (s->d_flag) (void)hipFree(s->d_flag);
  if (s->d_screen) (void)hipFree(s->d_screen);
  if (s->d_idx) (void)hipFree(s->d_idx);
  if (s->d_fc) (void)hipFree(s->d_fc);
  if (s->d_qc) (void)hipFree(s->d_qc);
  for (void* p : s->bufs) (void)hipFree(p);
  delete s;
  return EC_OK;
}

int ec_surrogate_num_params(const ec_surrogate* s, int64_t* n) {
  if (!s || !n) return set_error(EC_ERR_ARG, "null argument");
  *n = s->nparams;
  return EC_OK;
}

int ec_surrogate_get_params(const ec_surrogate* s, float* host) {
  if (!s || !host) return set_error(EC_ERR_ARG, "null argument");
  SCHK(hipMemcpy(host, s->d_p, s->nparams * sizeof(float), hipMemcpyDeviceToHost));
  return EC_OK;
}

int ec_surrogate_set_params(ec_surrogate* s, const float* host) {
  if (!s || !host) return set_error(EC_ERR_ARG, "null argument");
  SCHK(hipMemcpy(s->d_p, host, s->nparams * sizeof(float), hipMemcpyHostToDevice));
  s->adam_step = 0;
  SCHK(hipMemset(s->d_m, 0, s->nparams * sizeof(float)));
  SCHK(hipMemset(s->d_v, 0, s->nparams * sizeof(float)));
  return EC_OK;
}

int ec_surrogate_get_grads(const ec_surrogate* s, float* host) {
  if (!s || !host) return set_error(EC_ERR_ARG, "null argument");
  SCHK(hipMemcpy(host, s->d_g, s->nparams * sizeof(float), hipMemcpyDeviceToHost));
  return EC_OK;
}

int ec_surrogate_forward(ec_surrogate* s, const float* Fin, float* y, int B, void* stream) {
  return sguard([&]() -> int {
    if (!s || !Fin || !y) return set_error(EC_ERR_ARG, "null argument");
    if (B < 1 || B > s->maxB) return set_error(EC_ERR_ARG, "batch exceeds max_batch");
    hipStream_t st = (hipStream_t)stream;
    FnoArgs a = s->a;
    a.B = B;
    a.Fin = Fin;
    a.store_h = false;
    SCHK(fno_forward(a, st));
    SCHK(hipMemcpyAsync(y, a.y, (size_t)B * s->n * sizeof(float), hipMemcpyDeviceToDevice, st));
    return EC_OK;
  });
}

int ec_surrogate_train_step(ec_surrogate* s, const float* Fin, const float* target, int B,
                            float lr, int update, double* loss, void* stream) {
  return sguard([&]() -> int {
    if (!s || !Fin || !target) return set_error(EC_ERR_ARG, "null argument");
    if (B < 1 || B > s->maxB) return set_error(EC_ERR_ARG, "batch exceeds max_batch");
    hipStream_t st = (hipStream_t)stream;
    FnoArgs a = s->a;
    a.B = B;
    a.Fin = Fin;
    a.target = target;
    SCHK(fno_forward(a, st));
    SCHK(fno_backward(a, st));
    if (update) {
      s->adam_step += 1;
      SCHK(fno_adam(s->d_p, s->d_g, s->d_m, s->d_v, s->nparams, lr, 0.9f, 0.999f, 1e-8f,
                    s->adam_step, st));
    }
    if (loss) {
      std::vector<double> lb(B);
      SCHK(hipMemcpyAsync(lb.data(), a.loss_b, B * sizeof(double), hipMemcpyDeviceToHost, st));
      SCHK(hipStreamSynchronize(st));
      double acc = 0.0;
      for (double v : lb) acc += v;
      *loss = acc / B;
    }
    return EC_OK;
  });
}

int ec_surrogate_train(ec_surrogate* s, const float* Fin, const float* target, int B, float lr,
                       int update, double* loss, void* stream) {
  return ec_surrogate_train_step(s, Fin, target, B, lr, update, loss, stream);
}

int ec_surrogate_prepare(ec_surrogate* s, const ec_batch* batch, const double* f, const double* Q,
                         int64_t cell0, int B, float* Fin, float* target, void* stream) {
  return sguard([&]() -> int {
    if (!s || !batch || !f || !Fin) return set_error(EC_ERR_ARG, "null argument");
    if (B < 1 || cell0 < 0 || cell0 + B > batch_cells(batch))
      return set_error(EC_ERR_ARG, "cell range outside the batch");
    if (plan_N(batch_group_plan(batch, 0)) != s->N || plan_d(batch_group_plan(batch, 0)) != 3)
      return set_error(EC_ERR_ARG, "batch grid does not match the surrogate");
    if (B > s->maxB) return set_error(EC_ERR_ARG, "batch exceeds max_batch");
    hipStream_t st = (hipStream_t)stream;
    const double L = plan_L(batch_group_plan(batch, 0));
    const double h = 2.0 * L / s->N;
    SCHK(fno_normalize(f, batch_offsets_dev(batch), cell0, (int)s->n, h * h * h, B, s->d_red,
                       Fin, s->d_mass, st));
    if (Q && target)
      SCHK(fno_target(Q, batch_offsets_dev(batch), cell0, (int)s->n, B, s->d_mass, target, st));
    return EC_OK;
  });
}

int ec_surrogate_collide(ec_surrogate* s, ec_batch* batch, const double* f, double* Q,
                         double tau_m, double tau_e, int32_t* fell_back, double* screen,
                         int64_t* n_fallback, void* stream) {
  return sguard([&]() -> int {
    if (!s || !batch || !f || !Q) return set_error(EC_ERR_ARG, "null argument");
    if (f == Q) return set_error(EC_ERR_ARG, "f and Q must not alias");
    if (batch_groups(batch) != 1 || plan_N(batch_group_plan(batch, 0)) != s->N ||
        plan_d(batch_group_plan(batch, 0)) != 3)
      return set_error(EC_ERR_ARG, "the batch must be one group of 3D cells of the surrogate's N");
    hipStream_t st = (hipStream_t)stream;
    const int64_t ncell = batch_cells(batch);
    // screen buffers (the projection writes the residuals of every cell)
    if (!s->d_flag || s->scap < ncell) {
      if (s->d_flag) (void)hipFree(s->d_flag);
      if (s->d_screen) (void)hipFree(s->d_screen);
      if (s->d_idx) (void)hipFree(s->d_idx);
      s->d_flag = nullptr; s->d_screen = nullptr; s->d_idx = nullptr;
      s->scap = 0;
      if (hipMalloc(&s->d_flag, ncell * sizeof(int32_t)) != hipSuccess ||
          hipMalloc(&s->d_screen, ncell * 4 * sizeof(double)) != hipSuccess ||
          hipMalloc(&s->d_idx, ncell * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        if (s->d_flag) (void)hipFree(s->d_flag);
        if (s->d_screen) (void)hipFree(s->d_screen);
        s->d_flag = nullptr; s->d_screen = nullptr; s->d_idx = nullptr;
        return set_error(EC_ERR_OOM, "screen buffers");
      }
      s->scap = ncell;
    }
    for (int64_t c0 = 0; c0 < ncell; c0 += s->maxB) {
      const int B = (int)std::min<int64_t>(s->maxB, ncell - c0);
      int rc = forward_batch_cells(s, batch, f, Q, c0, B, st);
      if (rc) return rc;
    }
    // screen
    const double L = plan_L(batch_group_plan(batch, 0));
    hipLaunchKernelGGL(k_screen, dim3((unsigned)ncell), dim3(256), 0, st, f, Q,
                       batch_offsets_dev(batch), s->N, L, tau_m, tau_e, s->d_screen, s->d_flag);
    SCHK(hipGetLastError());
    std::vector<int32_t> flag(ncell);
    SCHK(hipMemcpyAsync(flag.data(), s->d_flag, ncell * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SCHK(hipStreamSynchronize(st));
    std::vector<int64_t> idx;
    for (int64_t c = 0; c < ncell; ++c)
      if (flag[c]) idx.push_back(c);
    if (fell_back) SCHK(hipMemcpyAsync(fell_back, s->d_flag, ncell * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    if (screen) SCHK(hipMemcpyAsync(screen, s->d_screen, ncell * 4 * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (n_fallback) *n_fallback = (int64_t)idx.size();
    const int64_t k = (int64_t)idx.size();
    if (k > 0) {
      // fallback batch of the same plan with capacity for every cell
      if (!s->fb || s->fb_cap < ncell) {
        if (s->fb) ec_batch_destroy(s->fb);
        s->fb = nullptr;
        if (s->d_fc) (void)hipFree(s->d_fc);
        if (s->d_qc) (void)hipFree(s->d_qc);
        s->d_fc = s->d_qc = nullptr;
        const ec_plan* plans[1] = {batch_group_plan(batch, 0)};
        int64_t counts[1] = {ncell};
        s->fb_cap = 0;
        int rc = ec_batch_create(plans, counts, 1, EC_FP64, &s->fb);
        if (rc) {
          s->fb = nullptr;
          return rc;
        }
        if (hipMalloc(&s->d_fc, batch_elems(s->fb) * sizeof(double)) != hipSuccess ||
            hipMalloc(&s->d_qc, batch_elems(s->fb) * sizeof(double)) != hipSuccess) {
          (void)hipGetLastError();
          if (s->d_fc) (void)hipFree(s->d_fc);
          s->d_fc = nullptr;
          ec_batch_destroy(s->fb);
          s->fb = nullptr;
          return set_error(EC_ERR_OOM, "fallback buffers");
        }
        s->fb_cap = ncell;   // only once every buffer of that capacity exists
      }
      SCHK(hipMemcpyAsync(s->d_idx, idx.data(), k * sizeof(int64_t), hipMemcpyHostToDevice, st));
      const int64_t tot = k * s->n;
      const unsigned g = (unsigned)((tot + 255) / 256);
      hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, st, f, batch_offsets_dev(batch), s->d_idx,
                         k, (int)s->n, batch_offsets_dev(s->fb), s->d_fc);
      SCHK(hipGetLastError());
      int rc = collide_prefix(s->fb, k, s->d_fc, s->d_qc, st);
      if (rc) return rc;
      hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, st, s->d_qc, batch_offsets_dev(s->fb),
                         s->d_idx, k, (int)s->n, batch_offsets_dev(batch), Q);
      SCHK(hipGetLastError());
      SCHK(hipStreamSynchronize(st));   // idx host vector goes out of scope
    }
    return EC_OK;
  });
}

}  // extern "C"

// C ABI of the EFM collision library (see include/ec.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/ec.h"
#include "fused.h"
#include "large2d.h"
#include "large3d.h"
#include "tables.h"
#include "internal.h"
#include "kernels.h"
#include "pipe.h"
#include "plan.h"

using namespace efm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(EC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename F>
int guarded(F&& fn) {
  try {
    return fn();
  } catch (const std::bad_alloc&) {
    return fail(EC_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(EC_ERR_ARG, e.what());
  } catch (...) {
    return fail(EC_ERR_ARG, "unknown exception");
  }
}

}  // namespace

namespace efm {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace efm

struct ec_plan {
  HostTables host;
  int device = 0;
  void* d_gamma64 = nullptr;   // [J][n] double pairs
  void* d_gamma32 = nullptr;   // [J][n] float pairs
  void* d_tw = nullptr;        // 2D grids of N >= 64: exp(2 pi i j / N), j < N
};

namespace {
bool is_large2d(const HostTables& T) { return T.d == 2 && large2d_supported(T.N); }
// 3D grids whose only schedule is the lines schedule (128^3)
bool is_large3d_only(const HostTables& T) { return T.d == 3 && T.N == 128; }
// plans that run in FP64 only (no FP32 copy of their tables is kept)
bool fp64_only(const HostTables& T) { return is_large2d(T) || is_large3d_only(T); }
bool lines_supported(const HostTables& T, int precision) {
  return T.d == 3 && large3d_supported(T.N) && precision == EC_FP64;
}
}  // namespace

struct BatchGroup {
  const ec_plan* plan = nullptr;
  int64_t count = 0;
  int64_t first = 0;   // first batch cell of the group
  int mode = 0;        // EC_SCHED_* (3D); 2D is always two-pass
  int chunk = 0;       // cells per pass / per pipeline chunk
  int G = 1;           // term groups (pipeline) or x split (fused)
};

struct StepGraph {
  hipGraphExec_t exec = nullptr;
  double* f = nullptr;
  double dt = 0.0;
  double* mon = nullptr;
  int method = 0;      // 0 forward Euler, 1 SSP-RK3
  int steps = 0;       // time steps recorded in the graph
};

// Most time steps one captured graph holds; longer runs launch it repeatedly
// (and a second graph for the remainder).
constexpr int kGraphMaxSteps = 200;

struct ProfRec {
  int group;
  int ncells;
  int kind;            // 0: two-pass chunk (3 kernels), 1: one pipeline launch, 2: fused chunk
  hipEvent_t ev[4];
};

struct ec_batch {
  bool profiling = false;
  std::vector<ProfRec> prof;        // recorded, not yet read
  std::vector<hipEvent_t> ev_pool;  // free events
  int precision = EC_FP64;
  int device = 0;
  std::vector<BatchGroup> groups;
  int64_t n_cells = 0, n_elems = 0;
  std::vector<int64_t> offsets;
  int64_t* d_off = nullptr;
  int* d_n = nullptr;
  double* d_hd = nullptr;
  int* d_geo = nullptr;     // per cell: N, d
  double* d_L = nullptr;    // per cell: L
  void* d_ws = nullptr;     // workspace shared by the groups (one at a time)
  size_t ws_bytes = 0;
  int* d_step = nullptr;
  StepGraph graph;          // kGraphMaxSteps steps (or all of a shorter run)
  StepGraph tail;           // the remainder of a longer run
  double* d_rk = nullptr;   // SSP-RK3 stage states: 2 x n_elems (allocated on first use)
};

namespace {

size_t csize(int precision) { return precision == EC_FP64 ? 16 : 8; }

// 32^3: split 4 (twice the workgroups of split 2, measured faster for 1 to
// 31 cells); otherwise the fused schedule's default split
int terms_default_split(int N, int precision) {
  return N == 32 ? 4 : fused_default_split(N, precision);
}

// Largest group that starts on the term-parallel schedule: its time grows
// with the cell count while the fused schedule's stays about flat until
// its workgroups fill the CUs; measured crossovers (FP64 / FP32): 16^3
// 192 / 192 cells, 24^3 64 / 80, 32^3 48 / 40.  0: no term-parallel default.
int64_t terms_default_max_cells(int N, int precision) {
  const bool fp64 = precision == EC_FP64;
  switch (N) {
    case 16: return 192;
    case 24: return fp64 ? 64 : 80;
    case 32: return fp64 ? 48 : 40;
    default: return 0;
  }
}

// Largest 2D group that starts on the term-parallel schedule (one block per
// (cell, term)).  Measured at 32^2, M = 16 (FP64, wall time per call):
// 1 cell 16 us against 101 us for the two-pass slab pass (one block walking
// every term), 64 cells 24 / 103 us, 1024 cells 101 / 118 us.
constexpr int64_t kTerms2dMaxCells = 1024;

// The term-parallel schedule exists for 3D N = 16, 24, 32 (FP64, FP32) and
// for the small 2D grids (two-pass sizes, FP64, FP32).
bool terms_ok(const HostTables& T, int precision) {
  if (T.d == 2)
    return T.N < 64 && terms_2d_supported(T.N) && precision != EC_BF16X3;
  return T.d == 3 && terms_supported(T.N, precision, terms_default_split(T.N, precision));
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return 256;
  return cus;
}

// Fused split for launches of `cells` cells: the default split, unless its
// workgroups (one per CU at these sizes) leave CUs idle in a launch that a
// larger split fills in one round (32^3: split 4 up to CUs / 4 cells), or
// need a second round that split 2 avoids (24^3: where 2 workgroups per
// cell fit one round over the CUs and 3 do not).  Measured on 256 CUs:
// 41-64 cells of 32^3 9-14 %
// (FP64) and 8-10 % (FP32) faster at split 4; 96 and 128 cells of 24^3 16 %
// and 13 % (FP64), 4-5 % (FP32) faster at split 2.
int fused_split_for(int N, int precision, int64_t cells) {
  const int d = fused_default_split(N, precision);
  if (d == 0) return 0;
  const int64_t cus = device_cus();
  if (N == 32 && 4 * cells <= cus) return 4;
  if (N == 24 && 2 * cells <= cus && 3 * cells > cus) return 2;
  return d;
}

void default_schedule(BatchGroup& g, int precision) {
  const HostTables& T = g.plan->host;
  const int64_t count = std::max<int64_t>(1, g.count);
  if (precision == EC_BF16X3) g.mode = EC_SCHED_TWO_PASS;   // the MFMA x pass is a separate kernel
  if (is_large3d_only(T)) g.mode = EC_SCHED_LINES;
  if (g.mode == EC_SCHED_LINES && !lines_supported(T, precision)) g.mode = EC_SCHED_TWO_PASS;
  if (g.mode == EC_SCHED_FUSED && (T.d != 3 || fused_default_split(T.N, precision) == 0))
    g.mode = EC_SCHED_TWO_PASS;
  if (g.mode == EC_SCHED_TERMS && !terms_ok(T, precision)) g.mode = EC_SCHED_PIPELINE;
  if (g.mode == EC_SCHED_PIPELINE && T.N > 32) g.mode = EC_SCHED_TWO_PASS;   // register lines <= 32
  if (T.d == 2 && g.mode == EC_SCHED_TERMS) {
    // per cell: the spectrum and J N^2 FP64 term partials; passes under ~2 GiB
    const double per_cell = (double)T.J * T.n * 8.0;
    const int64_t c = (int64_t)std::max(1.0, std::floor(2.0 * 1073741824.0 / per_cell));
    g.chunk = (int)std::max<int64_t>(1, std::min<int64_t>(c, count));
    g.G = 1;
  } else if (T.d == 3 && g.mode == EC_SCHED_TERMS) {
    // per cell: the half spectrum and J N^3 FP64 term partials; keep a pass
    // under ~2 GiB of partials
    const double per_cell = (double)T.J * T.n * 8.0;
    const int64_t c = (int64_t)std::max(1.0, std::floor(2.0 * 1073741824.0 / per_cell));
    g.chunk = (int)std::max<int64_t>(1, std::min<int64_t>(c, count));
    g.G = terms_default_split(T.N, precision);
  } else if (T.d == 3 && g.mode == EC_SCHED_FUSED) {
    // one spectrum per cell of workspace; 2048 cells keep >= 2048 workgroups busy
    g.chunk = (int)std::min<int64_t>(2048, count);
    g.G = fused_split_for(T.N, precision, g.chunk);
  } else if (T.d == 3 && g.mode == EC_SCHED_PIPELINE) {
    // keep one slot of the per-term intermediates under ~96 MB (the MALL holds
    // the slot being written and the slot being read), then split the terms so
    // the slab role has about 1024 blocks
    const double per_cell = (double)T.J * T.n * csize(precision);
    int64_t c = (int64_t)std::max(1.0, std::floor(96.0 * 1048576.0 / per_cell));
    g.chunk = (int)std::min<int64_t>(c, count);
    const int spb = (T.N == 24 || T.N == 12 ? 96 : 64) / T.N;
    const int64_t slab_blocks = ((int64_t)g.chunk * T.N + spb - 1) / spb;
    int G = (int)std::max<int64_t>(1, (1024 + slab_blocks - 1) / slab_blocks);
    g.G = std::min(G, std::min(T.J, 16));
  } else if (T.d == 3 && g.mode == EC_SCHED_LINES) {
    // per cell: spectrum and term volume (complex FP64) and the FP64
    // accumulator, 40 N^3 bytes; keep a pass under ~4 GiB of workspace
    const double per_cell = 40.0 * (double)T.n;
    const int64_t c = (int64_t)std::max(1.0, std::floor(4.0 * 1073741824.0 / per_cell));
    g.chunk = (int)std::max<int64_t>(1, std::min<int64_t>(c, count));
    g.G = 1;
  } else if (is_large2d(T)) {
    // per cell N^2 (spectrum) + J N^2 (per-term columns) complex FP64: keep a
    // pass under ~2 GiB of workspace
    const double per_cell = (double)(T.J + 1) * T.n * 16.0;
    const int64_t c = (int64_t)std::max(1.0, std::floor(2.0 * 1073741824.0 / per_cell));
    g.chunk = (int)std::max<int64_t>(1, std::min<int64_t>(c, count));
    g.G = 1;
  } else {
    // two-pass: aim for about 2048 waves in the slab pass (N0 * N threads per cell),
    // with the per-term intermediates of a pass under ~48 GiB (a sixth of HBM)
    const int64_t threads_per_cell = (int64_t)T.n0 * T.n1;
    int64_t c = (2048 * 64 + threads_per_cell - 1) / threads_per_cell;
    const double zcell = (double)(T.d == 3 ? T.J : 1) * T.n * csize(precision);
    c = std::min<int64_t>(c, (int64_t)std::max(1.0, std::floor(48.0 * 1073741824.0 / zcell)));
    g.chunk = (int)std::max<int64_t>(1, std::min<int64_t>(c, count));
    g.G = 1;
  }
}

bool use_pipe(const BatchGroup& g) { return g.plan->host.d == 3 && g.mode == EC_SCHED_PIPELINE; }
bool use_fused(const BatchGroup& g) { return g.plan->host.d == 3 && g.mode == EC_SCHED_FUSED; }
bool use_lines(const BatchGroup& g) { return g.plan->host.d == 3 && g.mode == EC_SCHED_LINES; }
bool use_terms(const BatchGroup& g) {
  return g.mode == EC_SCHED_TERMS && (g.plan->host.d == 3 || !is_large2d(g.plan->host));
}
bool fp32_tables(int precision) { return precision != EC_FP64; }

size_t group_ws_bytes(const BatchGroup& g, int precision) {
  const HostTables& T = g.plan->host;
  const size_t cs = csize(precision);
  const size_t n = (size_t)T.n;
  if (use_fused(g)) return (size_t)g.chunk * n * cs + 256;
  if (use_terms(g)) return (size_t)g.chunk * n * cs + 256 + (size_t)g.chunk * T.J * n * 8 + 256;
  if (use_lines(g)) return (size_t)g.chunk * n * 16 + 256 + (size_t)g.chunk * n * 24 + 256;
  if (use_pipe(g))
    return 2 * ((size_t)g.chunk * n * cs + (size_t)g.chunk * T.J * n * cs +
                (size_t)g.G * g.chunk * n * 8 + (size_t)g.chunk * n * 8) + 8 * 256;
  size_t bytes = (size_t)g.chunk * n * cs + 256;
  if (T.d == 3 || is_large2d(T)) bytes += (size_t)g.chunk * T.J * n * cs + 256;
  return bytes;
}

size_t batch_ws_bytes(const ec_batch* b) {
  size_t need = 0;
  for (auto& g : b->groups) need = std::max(need, group_ws_bytes(g, b->precision));
  return need;
}

// Sizes the shared workspace for the groups' current schedules.  The new
// buffer is allocated before the old one is released, so on failure the
// batch keeps a valid workspace of the old size (the caller restores the old
// schedules).  A buffer that is large enough is kept unless it is more than
// twice what is needed.
int alloc_workspaces(ec_batch* b) {
  const size_t need = batch_ws_bytes(b);
  if (b->d_ws && need <= b->ws_bytes && 2 * need >= b->ws_bytes) return EC_OK;
  if (need == 0) {
    if (b->d_ws) (void)hipFree(b->d_ws);
    b->d_ws = nullptr;
    b->ws_bytes = 0;
    return EC_OK;
  }
  void* p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess) {
    (void)hipGetLastError();
    if (b->d_ws && need <= b->ws_bytes) return EC_OK;   // the larger old buffer still serves
    return fail(EC_ERR_OOM, "workspace");
  }
  if (b->d_ws) (void)hipFree(b->d_ws);
  b->d_ws = p;
  b->ws_bytes = need;
  return EC_OK;
}

// Device memory that a schedule change could still obtain: what is free now
// (the old workspace stays allocated while the new one is created).
size_t device_free_bytes() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return (size_t)-1;
  }
  return fr;
}

char* align256(char* p) { return (char*)(((uintptr_t)p + 255) & ~(uintptr_t)255); }

void release_prof(ec_batch* b) {
  for (auto& r : b->prof)
    for (int k = 0; k < 4; ++k) b->ev_pool.push_back(r.ev[k]);
  b->prof.clear();
}

void drop_graph(ec_batch* b) {
  if (b->graph.exec) (void)hipGraphExecDestroy(b->graph.exec);
  if (b->tail.exec) (void)hipGraphExecDestroy(b->tail.exec);
  b->graph = StepGraph{};
  b->tail = StepGraph{};
}

hipEvent_t take_event(ec_batch* b) {
  if (!b->ev_pool.empty()) {
    hipEvent_t e = b->ev_pool.back();
    b->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int take_events(ec_batch* b, ProfRec& rec) {
  for (int k = 0; k < 4; ++k) {
    rec.ev[k] = take_event(b);
    if (!rec.ev[k]) return fail(EC_ERR_DEVICE, "hipEventCreate failed");
  }
  return EC_OK;
}

int run_group_two_pass(ec_batch* b, int gi, const double* f, double* Q, double dt,
                       hipStream_t s, bool profile) {
  const BatchGroup& g = b->groups[gi];
  const HostTables& T = g.plan->host;
  const size_t cs = csize(b->precision);
  char* W = align256((char*)b->d_ws);
  char* Z = align256(W + (size_t)g.chunk * T.n * cs);
  for (int64_t c0 = 0; c0 < g.count; c0 += g.chunk) {
    ChunkArgs a;
    a.N = T.N; a.d = T.d; a.precision = b->precision; a.J = T.J;
    a.gamma = fp32_tables(b->precision) ? g.plan->d_gamma32 : g.plan->d_gamma64;
    a.W = W; a.Z = (T.d == 3 || is_large2d(T)) ? Z : nullptr;
    a.f = f; a.Q = Q; a.off = b->d_off;
    a.cell0 = g.first + c0;
    a.ncells = (int)std::min<int64_t>(g.chunk, g.count - c0);
    a.dt = dt;
    a.tw = g.plan->d_tw;
    ProfRec rec{};
    if (profile) {
      rec.group = gi; rec.ncells = a.ncells; rec.kind = 0;
      int rc = take_events(b, rec);
      if (rc) return rc;
      a.ev = rec.ev;
    }
    if (is_large2d(T)) {
      HIPCHK(launch_large2d(a, a.tw, s));
    } else if (use_lines(g)) {
      HIPCHK(launch_large3d(a, a.tw, s));
    } else {
      HIPCHK(launch_chunk(a, s));
    }
    if (profile) b->prof.push_back(rec);
  }
  return EC_OK;
}

int run_group_pipe(ec_batch* b, int gi, const double* f, double* Q, double dt, hipStream_t s,
                   bool profile) {
  const BatchGroup& g = b->groups[gi];
  const HostTables& T = g.plan->host;
  const size_t cs = csize(b->precision);
  const size_t n = (size_t)T.n;
  PipeArgs base;
  base.gamma = fp32_tables(b->precision) ? g.plan->d_gamma32 : g.plan->d_gamma64;
  base.J = T.J; base.G = g.G; base.chunk = g.chunk;
  base.f = f; base.Q = Q; base.off = b->d_off; base.dt = dt;
  char* p = (char*)b->d_ws;
  for (int k = 0; k < 2; ++k) { p = align256(p); base.W[k] = p; p += (size_t)g.chunk * n * cs; }
  for (int k = 0; k < 2; ++k) { p = align256(p); base.Z[k] = p; p += (size_t)g.chunk * T.J * n * cs; }
  for (int k = 0; k < 2; ++k) { p = align256(p); base.Pg[k] = (double*)p; p += (size_t)g.G * g.chunk * n * 8; }
  for (int k = 0; k < 2; ++k) { p = align256(p); base.Lr[k] = (double*)p; p += (size_t)g.chunk * n * 8; }
  const int64_t nch = (g.count + g.chunk - 1) / g.chunk;
  auto cells_of = [&](int64_t k) { return (int)std::min<int64_t>(g.chunk, g.count - k * g.chunk); };
  for (int64_t i = 0; i < nch + 3; ++i) {
    PipeArgs a = base;
    if (i < nch) { a.f_cell0 = g.first + i * g.chunk; a.f_n = cells_of(i); a.f_slot = (int)(i & 1); }
    if (i - 1 >= 0 && i - 1 < nch) { a.p_cell0 = g.first + (i - 1) * g.chunk; a.p_n = cells_of(i - 1); a.p_slot = (int)((i - 1) & 1); }
    if (i - 2 >= 0 && i - 2 < nch) { a.s_cell0 = g.first + (i - 2) * g.chunk; a.s_n = cells_of(i - 2); a.s_slot = (int)((i - 2) & 1); }
    if (i - 3 >= 0 && i - 3 < nch) { a.c_cell0 = g.first + (i - 3) * g.chunk; a.c_n = cells_of(i - 3); a.c_slot = (int)((i - 3) & 1); }
    ProfRec rec{};
    if (profile) {
      rec.group = gi; rec.ncells = a.c_n; rec.kind = 1;
      int rc = take_events(b, rec);
      if (rc) return rc;
      HIPCHK(hipEventRecord(rec.ev[0], s));
    }
    HIPCHK(launch_pipe(a, T.N, b->precision, s));
    if (profile) {
      HIPCHK(hipEventRecord(rec.ev[3], s));
      b->prof.push_back(rec);
    }
  }
  return EC_OK;
}

int run_group_fused(ec_batch* b, int gi, const double* f, double* Q, double dt, hipStream_t s,
                    bool profile) {
  const BatchGroup& g = b->groups[gi];
  const HostTables& T = g.plan->host;
  char* W = align256((char*)b->d_ws);
  for (int64_t c0 = 0; c0 < g.count; c0 += g.chunk) {
    ChunkArgs a;
    a.N = T.N; a.d = T.d; a.precision = b->precision; a.J = T.J;
    a.gamma = fp32_tables(b->precision) ? g.plan->d_gamma32 : g.plan->d_gamma64;
    a.W = W;
    a.f = f; a.Q = Q; a.off = b->d_off;
    a.cell0 = g.first + c0;
    a.ncells = (int)std::min<int64_t>(g.chunk, g.count - c0);
    a.dt = dt;
    ProfRec rec{};
    if (profile) {
      rec.group = gi; rec.ncells = a.ncells; rec.kind = 2;
      int rc = take_events(b, rec);
      if (rc) return rc;
      a.ev = rec.ev;
    }
    HIPCHK(launch_fused(a, g.G, s));
    if (profile) b->prof.push_back(rec);
  }
  return EC_OK;
}

int run_group_terms(ec_batch* b, int gi, const double* f, double* Q, double dt, hipStream_t s,
                    bool profile) {
  const BatchGroup& g = b->groups[gi];
  const HostTables& T = g.plan->host;
  const size_t cs = csize(b->precision);
  char* W = align256((char*)b->d_ws);
  char* Zp = align256(W + (size_t)g.chunk * T.n * cs);
  for (int64_t c0 = 0; c0 < g.count; c0 += g.chunk) {
    ChunkArgs a;
    a.N = T.N; a.d = T.d; a.precision = b->precision; a.J = T.J;
    a.gamma = fp32_tables(b->precision) ? g.plan->d_gamma32 : g.plan->d_gamma64;
    a.W = W; a.Z = Zp;
    a.f = f; a.Q = Q; a.off = b->d_off;
    a.cell0 = g.first + c0;
    a.ncells = (int)std::min<int64_t>(g.chunk, g.count - c0);
    a.dt = dt;
    ProfRec rec{};
    if (profile) {
      rec.group = gi; rec.ncells = a.ncells; rec.kind = 2;
      int rc = take_events(b, rec);
      if (rc) return rc;
      a.ev = rec.ev;
    }
    HIPCHK(launch_terms(a, g.G, s));
    if (profile) b->prof.push_back(rec);
  }
  return EC_OK;
}

int run_group(ec_batch* b, int gi, const double* f, double* Q, double dt, hipStream_t s,
              bool profile) {
  const BatchGroup& g = b->groups[gi];
  if (use_fused(g)) return run_group_fused(b, gi, f, Q, dt, s, profile);
  if (use_terms(g)) return run_group_terms(b, gi, f, Q, dt, s, profile);
  if (use_pipe(g)) return run_group_pipe(b, gi, f, Q, dt, s, profile);
  return run_group_two_pass(b, gi, f, Q, dt, s, profile);
}

int run_collide(ec_batch* b, const double* f, double* Q, double dt, hipStream_t s,
                bool profile = false) {
  if (!b->d_ws && batch_ws_bytes(b) > 0)
    return fail(EC_ERR_OOM, "the batch has no workspace (an earlier allocation failed)");
  for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
    if (b->groups[gi].count == 0) continue;
    int rc = run_group(b, gi, f, Q, dt, s, profile);
    if (rc) return rc;
  }
  return EC_OK;
}

int check_batch_ptrs(ec_batch* b, const void* f, const void* Q) {
  if (!b) return fail(EC_ERR_ARG, "batch is null");
  if (!f) return fail(EC_ERR_ARG, "f is null");
  if (Q && f == Q) return fail(EC_ERR_ARG, "f and Q must not alias");
  return EC_OK;
}

}  // namespace

namespace efm {
const int64_t* batch_offsets_dev(const ec_batch* b) { return b->d_off; }
int64_t batch_cells(const ec_batch* b) { return b->n_cells; }
int64_t batch_elems(const ec_batch* b) { return b->n_elems; }
int batch_groups(const ec_batch* b) { return (int)b->groups.size(); }
const ec_plan* batch_group_plan(const ec_batch* b, int g) { return b->groups[g].plan; }
int64_t batch_group_count(const ec_batch* b, int g) { return b->groups[g].count; }
int plan_N(const ec_plan* p) { return p->host.N; }
int plan_d(const ec_plan* p) { return p->host.d; }
double plan_L(const ec_plan* p) { return p->host.L; }
int plan_J(const ec_plan* p) { return p->host.J; }
int plan_device(const ec_plan* p) { return p->device; }
const void* plan_gamma(const ec_plan* p, int precision) {
  return precision == EC_FP64 ? p->d_gamma64 : p->d_gamma32;
}
int fused_split_for_cells(int N, int precision, int64_t cells) {
  return fused_split_for(N, precision, cells);
}

int collide_prefix(ec_batch* b, int64_t n_active, const double* f, double* Q, hipStream_t s) {
  if (n_active <= 0) return EC_OK;
  BatchGroup& g = b->groups[0];
  const int64_t saved = g.count;
  g.count = std::min(saved, n_active);
  int rc = run_group(b, 0, f, Q, 0.0, s, false);
  g.count = saved;
  return rc;
}
}  // namespace efm

extern "C" {

const char* ec_last_error(void) { return g_err.c_str(); }

int ec_host_tables(int N, int d, double L, const ec_kernel* kernel, int M, int* n_terms,
                   double* gamma) {
  return guarded([&]() -> int {
    if (!kernel) return fail(EC_ERR_ARG, "kernel is null");
    HostTables T;
    std::string err;
    int rc = build_tables(N, d, L, kernel->kind, kernel->gamma, kernel->R, kernel->n_radial,
                          kernel->unfiltered, kernel->truncation, kernel->n_bcos,
                          kernel->bcos, M, T, err);
    if (rc) return fail(rc, err);
    if (n_terms) *n_terms = T.terms;
    if (gamma) std::memcpy(gamma, T.gamma.data(), T.gamma.size() * sizeof(double));
    return EC_OK;
  });
}

int ec_host_table_modes(int N, int d, double L, const ec_kernel* kernel, int M, int64_t n_modes,
                        const int64_t* modes, int* n_terms, double* gamma) {
  return guarded([&]() -> int {
    if (!kernel) return fail(EC_ERR_ARG, "kernel is null");
    if (n_modes < 0 || (n_modes > 0 && !modes)) return fail(EC_ERR_ARG, "bad mode list");
    HostTables T;
    std::vector<double> out;
    std::string err;
    int rc = build_table_modes(N, d, L, kernel->kind, kernel->gamma, kernel->R, kernel->n_radial,
                               kernel->unfiltered, kernel->truncation, kernel->n_bcos,
                               kernel->bcos, M, n_modes, modes, T, out, err);
    if (rc) return fail(rc, err);
    if (n_terms) *n_terms = T.terms;
    if (gamma) std::memcpy(gamma, out.data(), out.size() * sizeof(double));
    return EC_OK;
  });
}

int ec_setup_kernel(int N, int d, double L, const ec_kernel* kernel, int M, ec_plan** out) {
  return guarded([&]() -> int {
    if (!kernel || !out) return fail(EC_ERR_ARG, "null argument");
    *out = nullptr;
    auto* p = new ec_plan();
    std::string err;
    TableSpec spec;
    int rc = build_spec(N, d, L, kernel->kind, kernel->gamma, kernel->R, kernel->n_radial,
                        kernel->unfiltered, kernel->truncation, kernel->n_bcos, kernel->bcos, M,
                        p->host, spec, err);
    if (rc) { delete p; return fail(rc, err); }
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return fail(EC_ERR_DEVICE, "no HIP device"); }
    // the tables are filled on the device (the same per-mode formulas as the
    // host fill of ec_host_tables); no host copy is kept
    const size_t cnt = (size_t)2 * p->host.J * p->host.n;
    const bool with32 = !fp64_only(p->host);   // FP64-only plans keep no FP32 copy
    if (hipMalloc(&p->d_gamma64, cnt * sizeof(double)) != hipSuccess ||
        (with32 && hipMalloc(&p->d_gamma32, cnt * sizeof(float)) != hipSuccess)) {
      ec_plan_destroy(p);
      return fail(EC_ERR_OOM, "plan tables");
    }
    if (fill_tables_device(spec, (double*)p->d_gamma64, with32 ? (float*)p->d_gamma32 : nullptr) !=
        hipSuccess) {
      ec_plan_destroy(p);
      return fail(EC_ERR_DEVICE, "device fill of the plan tables failed");
    }
    if (is_large2d(p->host) || (p->host.d == 3 && large3d_supported(p->host.N))) {
      const std::vector<double> tw = twiddle_table(N);
      if (hipMalloc(&p->d_tw, tw.size() * sizeof(double)) != hipSuccess) {
        ec_plan_destroy(p);
        return fail(EC_ERR_OOM, "twiddle table");
      }
      if (hipMemcpy(p->d_tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        ec_plan_destroy(p);
        return fail(EC_ERR_DEVICE, "upload of the twiddle table failed");
      }
    }
    *out = p;
    return EC_OK;
  });
}

int ec_plan_destroy(ec_plan* p) {
  if (!p) return EC_OK;
  if (p->d_gamma64) (void)hipFree(p->d_gamma64);
  if (p->d_gamma32) (void)hipFree(p->d_gamma32);
  if (p->d_tw) (void)hipFree(p->d_tw);
  delete p;
  return EC_OK;
}

int ec_plan_terms(const ec_plan* p, int* n_terms) {
  if (!p || !n_terms) return fail(EC_ERR_ARG, "null argument");
  *n_terms = p->host.terms;
  return EC_OK;
}

int ec_plan_tables(const ec_plan* p, double* gamma) {
  if (!p || !gamma) return fail(EC_ERR_ARG, "null argument");
  HIPCHK(hipMemcpy(gamma, p->d_gamma64, (size_t)2 * p->host.J * p->host.n * sizeof(double),
                   hipMemcpyDeviceToHost));
  return EC_OK;
}

int ec_batch_create(const ec_plan* const* plans, const int64_t* counts, int n_groups,
                    int precision, ec_batch** out) {
  return guarded([&]() -> int {
    if (!plans || !counts || !out || n_groups < 1) return fail(EC_ERR_ARG, "null argument or no groups");
    if (precision != EC_FP64 && precision != EC_FP32 && precision != EC_BF16X3)
      return fail(EC_ERR_ARG, "precision");
    if (precision == EC_BF16X3)
      for (int g = 0; g < n_groups; ++g)
        if (plans[g] && counts[g] > 0 &&
            !(plans[g]->host.d == 3 &&
              (plans[g]->host.N == 16 || plans[g]->host.N == 32 || plans[g]->host.N == 64)))
          return fail(EC_ERR_UNSUPPORTED, "split-BF16 transforms need 3D cells with N = 16, 32 or 64");
    if (precision != EC_FP64)
      for (int g = 0; g < n_groups; ++g)
        if (plans[g] && counts[g] > 0 && fp64_only(plans[g]->host))
          return fail(EC_ERR_UNSUPPORTED, "2D grids of N >= 64 and 3D grids of N = 128 are FP64 only");
    *out = nullptr;
    auto* b = new ec_batch();
    b->precision = precision;
    if (hipGetDevice(&b->device) != hipSuccess) { delete b; return fail(EC_ERR_DEVICE, "no HIP device"); }
    int64_t cell = 0, elem = 0;
    std::vector<int> ns, geo;
    std::vector<double> hds, Ls;
    for (int g = 0; g < n_groups; ++g) {
      if (!plans[g] || counts[g] < 0) { delete b; return fail(EC_ERR_ARG, "bad group"); }
      BatchGroup bg;
      bg.plan = plans[g];
      bg.count = counts[g];
      bg.first = cell;
      // the fused schedule runs P workgroups per cell: for small groups the
      // term-parallel form (J P workgroups per cell) fills more CUs.  Small
      // groups of other sizes take the pipelined schedule (term groups
      // spread one cell over many workgroups); each falls back to two-pass
      // where absent
      const int64_t tmax = plans[g]->host.d == 2
                               ? kTerms2dMaxCells
                               : terms_default_max_cells(plans[g]->host.N, precision);
      bg.mode = counts[g] <= tmax ? EC_SCHED_TERMS
                                  : (counts[g] >= 32 ? EC_SCHED_FUSED : EC_SCHED_PIPELINE);
      default_schedule(bg, precision);
      const HostTables& T = plans[g]->host;
      const double hd = std::pow(2.0 * T.L / T.N, T.d);
      for (int64_t c = 0; c < counts[g]; ++c) {
        b->offsets.push_back(elem);
        ns.push_back((int)T.n);
        hds.push_back(hd);
        geo.push_back(T.N);
        geo.push_back(T.d);
        Ls.push_back(T.L);
        elem += (T.n + 31) / 32 * 32;   // 256-byte aligned cells
      }
      cell += counts[g];
      b->groups.push_back(bg);
    }
    b->n_cells = cell;
    b->n_elems = elem;
    if (cell > 0) {
      if (hipMalloc(&b->d_off, cell * sizeof(int64_t)) != hipSuccess ||
          hipMalloc(&b->d_n, cell * sizeof(int)) != hipSuccess ||
          hipMalloc(&b->d_hd, cell * sizeof(double)) != hipSuccess ||
          hipMalloc(&b->d_geo, 2 * cell * sizeof(int)) != hipSuccess ||
          hipMalloc(&b->d_L, cell * sizeof(double)) != hipSuccess) {
        ec_batch_destroy(b);
        return fail(EC_ERR_OOM, "batch metadata");
      }
      if (hipMemcpy(b->d_off, b->offsets.data(), cell * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(b->d_n, ns.data(), cell * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(b->d_hd, hds.data(), cell * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(b->d_geo, geo.data(), 2 * cell * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(b->d_L, Ls.data(), cell * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        ec_batch_destroy(b);
        return fail(EC_ERR_DEVICE, "upload of batch metadata failed");
      }
    }
    if (hipMalloc(&b->d_step, 2 * sizeof(int)) != hipSuccess) { ec_batch_destroy(b); return fail(EC_ERR_OOM, "step counter"); }
    int rc = alloc_workspaces(b);
    if (rc) { ec_batch_destroy(b); return rc; }
    *out = b;
    return EC_OK;
  });
}

int ec_batch_destroy(ec_batch* b) {
  if (!b) return EC_OK;
  drop_graph(b);
  release_prof(b);
  for (auto e : b->ev_pool) (void)hipEventDestroy(e);
  if (b->d_off) (void)hipFree(b->d_off);
  if (b->d_n) (void)hipFree(b->d_n);
  if (b->d_hd) (void)hipFree(b->d_hd);
  if (b->d_geo) (void)hipFree(b->d_geo);
  if (b->d_L) (void)hipFree(b->d_L);
  if (b->d_ws) (void)hipFree(b->d_ws);
  if (b->d_step) (void)hipFree(b->d_step);
  if (b->d_rk) (void)hipFree(b->d_rk);
  delete b;
  return EC_OK;
}

int ec_batch_size(const ec_batch* b, int64_t* n_cells, int64_t* n_elems) {
  if (!b) return fail(EC_ERR_ARG, "batch is null");
  if (n_cells) *n_cells = b->n_cells;
  if (n_elems) *n_elems = b->n_elems;
  return EC_OK;
}

int ec_batch_offsets(const ec_batch* b, int64_t* offsets) {
  if (!b || !offsets) return fail(EC_ERR_ARG, "null argument");
  std::memcpy(offsets, b->offsets.data(), b->offsets.size() * sizeof(int64_t));
  return EC_OK;
}

int ec_batch_set_schedule(ec_batch* b, int group, int mode, int cells_per_pass, int term_groups) {
  return guarded([&]() -> int {
    if (!b || group < 0 || group >= (int)b->groups.size()) return fail(EC_ERR_ARG, "bad group");
    if (mode != EC_SCHED_PIPELINE && mode != EC_SCHED_TWO_PASS && mode != EC_SCHED_FUSED &&
        mode != EC_SCHED_LINES && mode != EC_SCHED_TERMS)
      return fail(EC_ERR_ARG, "bad mode");
    BatchGroup& g = b->groups[group];
    const BatchGroup saved = g;
    auto restore = [&](int rc) {
      g = saved;
      return rc;
    };
    if (mode == EC_SCHED_TERMS && !terms_ok(g.plan->host, b->precision))
      return fail(EC_ERR_UNSUPPORTED,
                  "the term-parallel schedule needs 3D cells of N = 16, 24 or 32 or 2D cells of "
                  "N <= 32, in FP64 or FP32");
    if (mode == EC_SCHED_LINES && !lines_supported(g.plan->host, b->precision))
      return fail(EC_ERR_UNSUPPORTED, "the lines schedule needs 3D cells of N = 64 or 128 in FP64");
    if (mode != EC_SCHED_LINES && is_large3d_only(g.plan->host))
      return fail(EC_ERR_UNSUPPORTED, "128^3 grids run only the lines schedule");
    g.mode = mode;
    default_schedule(g, b->precision);
    const int64_t count = std::max<int64_t>(1, g.count);
    if (cells_per_pass > 0) g.chunk = (int)std::min<int64_t>(cells_per_pass, count);
    if (term_groups > 0 && use_pipe(g)) g.G = std::min(term_groups, g.plan->host.J);
    if (term_groups > 0 && use_fused(g)) {
      if (!fused_supported(g.plan->host.N, b->precision, term_groups))
        return restore(fail(EC_ERR_UNSUPPORTED, "unsupported x split for the fused schedule"));
      g.G = term_groups;
    }
    if (term_groups > 0 && use_terms(g)) {
      if (!terms_supported(g.plan->host.N, b->precision, term_groups))
        return restore(fail(EC_ERR_UNSUPPORTED, "unsupported x split for the term-parallel schedule"));
      g.G = term_groups;
    }
    drop_graph(b);
    if (hipDeviceSynchronize() != hipSuccess) return restore(fail(EC_ERR_DEVICE, "device sync failed"));
    const int rc = alloc_workspaces(b);
    return rc ? restore(rc) : EC_OK;
  });
}

int ec_batch_set_chunk(ec_batch* b, int group, int cells_per_pass) {
  if (!b || group < 0 || group >= (int)b->groups.size()) return fail(EC_ERR_ARG, "bad group");
  return ec_batch_set_schedule(b, group, b->groups[group].mode, cells_per_pass, 0);
}

int ec_batch_get_schedule(const ec_batch* b, int group, int* mode, int* cells_per_pass,
                          int* term_groups) {
  if (!b || group < 0 || group >= (int)b->groups.size()) return fail(EC_ERR_ARG, "bad group");
  const BatchGroup& g = b->groups[group];
  if (mode)
    *mode = use_fused(g)   ? EC_SCHED_FUSED
            : use_terms(g) ? EC_SCHED_TERMS
            : use_pipe(g)  ? EC_SCHED_PIPELINE
            : use_lines(g) ? EC_SCHED_LINES
                           : EC_SCHED_TWO_PASS;
  if (cells_per_pass) *cells_per_pass = g.chunk;
  if (term_groups) *term_groups = g.G;
  return EC_OK;
}

int ec_collide(ec_batch* b, const double* f, double* Q, void* stream) {
  return guarded([&]() -> int {
    int rc = check_batch_ptrs(b, f, Q);
    if (rc) return rc;
    if (!Q) return fail(EC_ERR_ARG, "Q is null");
    return run_collide(b, f, Q, 0.0, (hipStream_t)stream, b->profiling);
  });
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
namespace {

struct Sched {
  int mode, chunk, G;
};

std::string tune_key(int dev, const HostTables& T, int precision, int64_t count) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|d%d|N%d|M%d|kind%d|L%.6g|R%.6g|prec%d|cells%lld", arch.c_str(),
                T.d, T.N, T.M, T.kind, T.L, T.R, precision, (long long)count);
  std::string key = buf;
  if (T.n_radial > 1) {   // non-separable kernels: exponent and radial nodes too
    std::snprintf(buf, sizeof buf, "|g%.6g|nr%d", T.gamma_exp, T.n_radial);
    key += buf;
  }
  if (T.unfiltered) key += "|nofilter";
  if (T.truncation == EC_TRUNC_BALL) key += "|ball";
  for (size_t i = 0; i < T.bcos.size(); ++i) {
    std::snprintf(buf, sizeof buf, "%sb%.6g", i ? "," : "|", T.bcos[i]);
    key += buf;
  }
  return key;
}

// cache format: one line per key, "<key> <mode> <chunk> <G> <ms>"
bool cache_lookup(const char* path, const std::string& key, Sched& out) {
  if (!path || !*path) return false;
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string k;
    Sched s{};
    double ms;
    if (ls >> k >> s.mode >> s.chunk >> s.G >> ms && k == key) { out = s; found = true; }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const Sched& s, double ms) {
  if (!path || !*path) return;
  std::ofstream outf(path, std::ios::app);
  if (outf) outf << key << ' ' << s.mode << ' ' << s.chunk << ' ' << s.G << ' ' << ms << '\n';
}

// Workspace bytes the batch would need with group gi on schedule s.
size_t sched_ws_bytes(const ec_batch* b, int gi, const Sched& s) {
  BatchGroup g = b->groups[gi];
  g.mode = s.mode;
  default_schedule(g, b->precision);
  const int64_t count = std::max<int64_t>(1, g.count);
  if (s.chunk > 0) g.chunk = (int)std::min<int64_t>(s.chunk, count);
  if (s.G > 0 && use_pipe(g)) g.G = std::min(s.G, g.plan->host.J);
  size_t need = group_ws_bytes(g, b->precision);
  for (int i = 0; i < (int)b->groups.size(); ++i)
    if (i != gi) need = std::max(need, group_ws_bytes(b->groups[i], b->precision));
  return need;
}

int apply_sched(ec_batch* b, int gi, const Sched& s) {
  BatchGroup& g = b->groups[gi];
  const BatchGroup saved = g;
  g.mode = s.mode;
  default_schedule(g, b->precision);
  const int64_t count = std::max<int64_t>(1, g.count);
  if (s.chunk > 0) g.chunk = (int)std::min<int64_t>(s.chunk, count);
  if (s.G > 0 && use_pipe(g)) g.G = std::min(s.G, g.plan->host.J);
  if (s.G > 0 && use_fused(g) && fused_supported(g.plan->host.N, b->precision, s.G)) g.G = s.G;
  if (s.G > 0 && use_terms(g) && terms_supported(g.plan->host.N, b->precision, s.G)) g.G = s.G;
  const int rc = alloc_workspaces(b);
  if (rc) g = saved;
  return rc;
}

int time_group(ec_batch* b, int gi, const double* f, double* Q, hipStream_t st, double& best_ms) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  best_ms = 1e30;
  int rc = EC_OK;
  for (int r = 0; r < 4 && rc == EC_OK; ++r) {
    (void)hipEventRecord(e0, st);
    rc = run_group(b, gi, f, Q, 0.0, st, false);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) rc = fail(EC_ERR_DEVICE, "autotune run failed");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (r > 0) best_ms = std::min(best_ms, (double)ms);   // first run is a warm-up
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

int ec_autotune(ec_batch* b, const double* f, double* Q, const char* cache_path, int flags,
                void* stream) {
  return guarded([&]() -> int {
    int rc = check_batch_ptrs(b, f, Q);
    if (rc) return rc;
    if (!Q) return fail(EC_ERR_ARG, "Q is null");
    hipStream_t st = (hipStream_t)stream;
    drop_graph(b);
    for (int gi = 0; gi < (int)b->groups.size(); ++gi) {
      BatchGroup& g = b->groups[gi];
      if (g.count == 0) continue;
      const HostTables& T = g.plan->host;
      const std::string key = tune_key(b->device, T, b->precision, g.count);
      Sched best{};
      if (!(flags & EC_TUNE_REMEASURE) && cache_lookup(cache_path, key, best)) {
        rc = apply_sched(b, gi, best);
        if (rc) return rc;
        continue;
      }
      std::vector<Sched> cand;
      const int64_t count = g.count;
      if (lines_supported(T, b->precision))
        for (int c : {1, 4, 16, 64}) {
          const Sched sl{EC_SCHED_LINES, (int)std::min<int64_t>(c, count), 0};
          bool dup = false;
          for (auto& x : cand) dup |= (x.mode == sl.mode && x.chunk == sl.chunk);
          if (!dup) cand.push_back(sl);
        }
      for (int c : {16, 32, 64, 128, 256, 1024, 4096}) {
        if (is_large3d_only(T)) break;
        Sched s{EC_SCHED_TWO_PASS, (int)std::min<int64_t>(c, count), 0};
        bool dup = false;
        for (auto& x : cand) dup |= (x.mode == s.mode && x.chunk == s.chunk);
        if (!dup) cand.push_back(s);
      }
      if (T.d == 3 && fused_default_split(T.N, b->precision) > 0) {
        for (int P : {1, 2, 3, 4})
          if (fused_supported(T.N, b->precision, P))
            for (int c : {256, 512, 1024, 2048}) {
              const Sched sc{EC_SCHED_FUSED, (int)std::min<int64_t>(c, count), P};
              bool dup = false;
              for (auto& x : cand) dup |= (x.mode == sc.mode && x.chunk == sc.chunk && x.G == sc.G);
              if (!dup) cand.push_back(sc);
            }
      }
      if (T.d == 2 && count < 256 && terms_ok(T, b->precision)) {
        BatchGroup probe = g;
        probe.mode = EC_SCHED_TERMS;
        default_schedule(probe, b->precision);
        cand.push_back(Sched{EC_SCHED_TERMS, probe.chunk, 1});
      }
      if (T.d == 3 && count < 256 &&
          terms_supported(T.N, b->precision, terms_default_split(T.N, b->precision))) {
        BatchGroup probe = g;
        probe.mode = EC_SCHED_TERMS;
        default_schedule(probe, b->precision);
        for (int P : {1, 2, 3, 4})
          if (terms_supported(T.N, b->precision, P))
            cand.push_back(Sched{EC_SCHED_TERMS, probe.chunk, P});
      }
      if (T.d == 3 && T.N <= 32) {
        for (int c : {4, 6, 8, 12, 16, 24})
          for (int G : {1, 2, 4, 8}) {
            if (c > count && c != 4) continue;
            cand.push_back(Sched{EC_SCHED_PIPELINE, (int)std::min<int64_t>(c, count), G});
          }
      }
      // keep a margin of 1/16 of the free memory for the caller; a
      // candidate whose workspace does not fit is not measured
      const size_t room = std::max(b->ws_bytes, device_free_bytes() / 16 * 15);
      std::vector<Sched> fit;
      for (auto& s : cand)
        if (sched_ws_bytes(b, gi, s) <= room) fit.push_back(s);
      if (fit.empty()) return fail(EC_ERR_OOM, "no schedule's workspace fits the free device memory");
      double best_ms = 1e30;
      best = fit[0];
      for (auto& s : fit) {
        rc = apply_sched(b, gi, s);
        if (rc == EC_ERR_OOM) continue;   // the old schedule and workspace are kept
        if (rc) return rc;
        double ms;
        rc = time_group(b, gi, f, Q, st, ms);
        if (rc) return rc;
        if (ms < best_ms) { best_ms = ms; best = s; }
      }
      if (best_ms >= 1e30) return fail(EC_ERR_OOM, "no candidate schedule's workspace could be allocated");
      rc = apply_sched(b, gi, best);
      if (rc) return rc;
      cache_store(cache_path, key, best, best_ms);
    }
    return EC_OK;
  });
}

int ec_copy(const double* src, double* dst, int64_t n, void* stream) {
  if (!src || !dst || n < 0) return fail(EC_ERR_ARG, "bad copy arguments");
  HIPCHK(launch_copy(src, dst, n, (hipStream_t)stream));
  return EC_OK;
}

int ec_valu_probe(int precision, double* tflops, void* stream) {
  return guarded([&]() -> int {
    if (!tflops || (precision != EC_FP64 && precision != EC_FP32))
      return fail(EC_ERR_ARG, "bad probe arguments");
    hipStream_t st = (hipStream_t)stream;
    const int blocks = 8192, iters = 2048;
    void* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (sink) (void)hipFree(sink);
    };
    if (hipMalloc(&sink, sizeof(double)) != hipSuccess) return fail(EC_ERR_OOM, "probe sink");
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      cleanup();
      return fail(EC_ERR_DEVICE, "probe events");
    }
    // two warm-up launches, then the fastest of five timed ones (the clock
    // settles under load)
    hipError_t e = launch_valu_probe(precision, blocks, iters, sink, st);
    if (e == hipSuccess) e = launch_valu_probe(precision, blocks, iters, sink, st);
    float ms = 0.f;
    for (int rep = 0; rep < 5 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = launch_valu_probe(precision, blocks, iters, sink, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e == hipSuccess && (rep == 0 || t < ms)) ms = t;
    }
    cleanup();
    if (e != hipSuccess) return fail(EC_ERR_DEVICE, hipGetErrorString(e));
    const double flops = 2.0 * blocks * 256.0 * iters * valu_probe_chains();
    *tflops = ms > 0.f ? flops / (ms * 1e-3) / 1e12 : 0.0;
    return EC_OK;
  });
}

int ec_profile(ec_batch* b, int enable) {
  if (!b) return fail(EC_ERR_ARG, "batch is null");
  b->profiling = enable != 0;
  return EC_OK;
}

int ec_profile_read(ec_batch* b, double* ms, int64_t* launches, int64_t* cells) {
  return guarded([&]() -> int {
    if (!b || !ms || !launches || !cells) return fail(EC_ERR_ARG, "null argument");
    const int G = (int)b->groups.size();
    for (int i = 0; i < EC_PROF_KERNELS * G; ++i) { ms[i] = 0.0; launches[i] = 0; }
    for (int g = 0; g < G; ++g) cells[g] = 0;
    for (auto& r : b->prof) {
      HIPCHK(hipEventSynchronize(r.ev[3]));
      if (r.kind == 0) {
        for (int k = 0; k < 3; ++k) {
          float t = 0.f;
          HIPCHK(hipEventElapsedTime(&t, r.ev[k], r.ev[k + 1]));
          ms[EC_PROF_KERNELS * r.group + k] += t;
          launches[EC_PROF_KERNELS * r.group + k] += 1;
        }
      } else if (r.kind == 2) {
        // the forward transform (events 0 -> 1) and the fused or term kernels
        // (2 -> 3); 1 -> 2 is empty
        const int slot[2] = {0, 5}, from[2] = {0, 2}, to[2] = {1, 3};
        for (int k = 0; k < 2; ++k) {
          float t = 0.f;
          HIPCHK(hipEventElapsedTime(&t, r.ev[from[k]], r.ev[to[k]]));
          ms[EC_PROF_KERNELS * r.group + slot[k]] += t;
          launches[EC_PROF_KERNELS * r.group + slot[k]] += 1;
        }
      } else {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, r.ev[0], r.ev[3]));
        ms[EC_PROF_KERNELS * r.group + 3] += t;
        launches[EC_PROF_KERNELS * r.group + 3] += 1;
      }
      cells[r.group] += r.ncells;
    }
    release_prof(b);
    return EC_OK;
  });
}

int ec_entropy_prod(ec_batch* b, const double* f, const double* Q, double* out,
                    int32_t* n_nonpos, void* stream) {
  return guarded([&]() -> int {
    int rc = check_batch_ptrs(b, f, Q);
    if (rc) return rc;
    if (!Q || !out) return fail(EC_ERR_ARG, "Q or out is null");
    HIPCHK(launch_monitors(f, Q, b->d_off, b->d_n, b->d_hd, b->d_geo, b->d_L, 0, b->n_cells, nullptr, out,
                           n_nonpos, nullptr, nullptr, 0, nullptr, (hipStream_t)stream));
    return EC_OK;
  });
}

int ec_monitors(ec_batch* b, const double* f, const double* Q, double* out, void* stream) {
  return guarded([&]() -> int {
    int rc = check_batch_ptrs(b, f, Q);
    if (rc) return rc;
    if (!out) return fail(EC_ERR_ARG, "out is null");
    HIPCHK(launch_monitors(f, Q, b->d_off, b->d_n, b->d_hd, b->d_geo, b->d_L, 0, b->n_cells, out, nullptr,
                           nullptr, nullptr, nullptr, 0, nullptr, (hipStream_t)stream));
    return EC_OK;
  });
}

}  // extern "C"

namespace {

// One time step of `method` on f in place, recorded on stream s (captured).
int record_step(ec_batch* b, double* f, double dt, int method, double* monitors, hipStream_t s) {
  int rc = EC_OK;
  if (method == 0) {
    rc = run_collide(b, f, f, dt, s);
  } else {
    // Shu-Osher form: u1 = f + dt Q(f); u2 = 3/4 f + 1/4 (u1 + dt Q(u1));
    // f <- 1/3 f + 2/3 (u2 + dt Q(u2)).  u1 and u2 share a buffer.
    double* u = b->d_rk;
    double* w = b->d_rk + b->n_elems;
    rc = run_collide(b, f, u, dt, s);
    if (rc == EC_OK) rc = run_collide(b, u, w, dt, s);
    if (rc == EC_OK) {
      hipError_t e = launch_axpby_cells(f, w, u, 0.75, 0.25, b->d_off, b->d_n, b->n_cells, s);
      if (e != hipSuccess) rc = fail(EC_ERR_DEVICE, hipGetErrorString(e));
    }
    if (rc == EC_OK) rc = run_collide(b, u, w, dt, s);
    if (rc == EC_OK) {
      hipError_t e = launch_axpby_cells(f, w, f, 1.0 / 3.0, 2.0 / 3.0, b->d_off, b->d_n,
                                        b->n_cells, s);
      if (e != hipSuccess) rc = fail(EC_ERR_DEVICE, hipGetErrorString(e));
    }
  }
  if (rc == EC_OK && monitors) {
    hipError_t e2 = launch_monitors(f, nullptr, b->d_off, b->d_n, b->d_hd, b->d_geo, b->d_L, 0, b->n_cells, nullptr,
                                    nullptr, nullptr, b->d_step, monitors, b->n_cells,
                                    b->d_step + 1, s);
    if (e2 == hipSuccess) e2 = launch_inc_int(b->d_step, s);
    if (e2 != hipSuccess) rc = fail(EC_ERR_DEVICE, hipGetErrorString(e2));
  }
  return rc;
}

// Captures `steps` consecutive time steps into one graph (g), unless g
// already holds exactly that.
int capture_steps(ec_batch* b, StepGraph& g, double* f, double dt, double* monitors, int method,
                  int steps) {
  if (g.exec && g.f == f && g.dt == dt && g.mon == monitors && g.method == method &&
      g.steps == steps)
    return EC_OK;
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g = StepGraph{};
  hipStream_t cap_stream;
  HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal);
  int rc = EC_OK;
  if (e == hipSuccess) {
    for (int k = 0; k < steps && rc == EC_OK; ++k)
      rc = record_step(b, f, dt, method, monitors, cap_stream);
    hipError_t e3 = hipStreamEndCapture(cap_stream, &graph);
    if (rc == EC_OK && e3 != hipSuccess) rc = fail(EC_ERR_DEVICE, hipGetErrorString(e3));
  } else {
    rc = fail(EC_ERR_DEVICE, hipGetErrorString(e));
  }
  if (rc == EC_OK) {
    hipError_t e4 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e4 != hipSuccess) {
      g.exec = nullptr;
      rc = fail(EC_ERR_DEVICE, hipGetErrorString(e4));
    }
  }
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap_stream);
  if (rc) return rc;
  g.f = f;
  g.dt = dt;
  g.mon = monitors;
  g.method = method;
  g.steps = steps;
  return EC_OK;
}

int run_steps(ec_batch* b, double* f, double dt, int n_steps, double* monitors, int method,
              hipStream_t s) {
  if (n_steps < 0 || !(dt > 0.0)) return fail(EC_ERR_ARG, "need dt > 0 and n_steps >= 0");
  if (n_steps == 0) return EC_OK;
  if (!b->d_ws && batch_ws_bytes(b) > 0)
    return fail(EC_ERR_OOM, "the batch has no workspace (an earlier allocation failed)");
  if (method == 1 && !b->d_rk) {
    HIPCHK(hipDeviceSynchronize());
    void* p = nullptr;
    if (hipMalloc(&p, 2 * (size_t)b->n_elems * sizeof(double)) != hipSuccess)
      return fail(EC_ERR_OOM, "SSP-RK3 stage buffers");
    b->d_rk = (double*)p;
  }
  // up to kGraphMaxSteps steps in one graph; a longer run launches it
  // repeatedly and a second graph for the remainder
  const int K = std::min(n_steps, kGraphMaxSteps);
  const int full = n_steps / K, rest = n_steps % K;
  int rc = capture_steps(b, b->graph, f, dt, monitors, method, K);
  if (rc == EC_OK && rest) rc = capture_steps(b, b->tail, f, dt, monitors, method, rest);
  if (rc) {
    drop_graph(b);
    return rc;
  }
  // step counter and the capacity of the monitor buffer (in steps)
  HIPCHK(launch_set_int(b->d_step, 0, s));
  HIPCHK(launch_set_int(b->d_step + 1, monitors ? n_steps : 0, s));
  for (int k = 0; k < full; ++k) HIPCHK(hipGraphLaunch(b->graph.exec, s));
  if (rest) HIPCHK(hipGraphLaunch(b->tail.exec, s));
  return EC_OK;
}

}  // namespace

extern "C" {

int ec_step(ec_batch* b, double* f, double dt, int n_steps, double* monitors, void* stream) {
  return guarded([&]() -> int {
    int rc = check_batch_ptrs(b, f, nullptr);
    if (rc) return rc;
    return run_steps(b, f, dt, n_steps, monitors, 0, (hipStream_t)stream);
  });
}

int ec_step_graph(ec_batch* b, double* f, double dt, int n_steps, double* monitors,
                  void* stream) {
  return ec_step(b, f, dt, n_steps, monitors, stream);
}

int ec_step_ssprk3(ec_batch* b, double* f, double dt, int n_steps, double* monitors,
                   void* stream) {
  return guarded([&]() -> int {
    int rc = check_batch_ptrs(b, f, nullptr);
    if (rc) return rc;
    return run_steps(b, f, dt, n_steps, monitors, 1, (hipStream_t)stream);
  });
}

}  // extern "C"

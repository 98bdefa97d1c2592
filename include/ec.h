/*
 * ec.h -- C ABI of the MI355X library for the entropic Fourier method (EFM)
 * collision operator (Z. Cai, Y. Fan, L. Ying, "An entropic Fourier method for
 * the Boltzmann equation", arXiv 1704.07369).
 *
 * The library evaluates, for many independent space-homogeneous cells, the
 * discrete collision term
 *
 *     Q_r = sum_{l,m in K} (B^s(l,m) - B^s(m,m)) Fh_l Fh_m E_{l+m}(r),  r in X
 *
 * (section 3.2.2, eq. Qsk / eq. Qsr) with the filtered low-rank kernel modes of
 * the fast algorithm (section 4.1, eq. fastAlg and its filtered form), by
 * 2 M' + 2 FFTs per cell: one forward transform, M' inverse transforms of
 * (alpha_t + i beta_t) Fh (the gain sum_t a_t b_t, section 3.3), and one
 * inverse transform of the diagonal multiplier (the loss F_r l_r, section
 * 3.1.2).
 *
 * Conventions (the input contract of section 3.3, eq. I_N):
 *  - velocity box [-L, L]^d, N points per axis, h = 2L/N, v_j = -L + j h;
 *  - a cell is N^d FP64 point samples F_r = f(v_r) >= 0, C order, last axis
 *    fastest;
 *  - all device pointers are owned by the caller; the library owns only its
 *    plans, batches and their workspaces;
 *  - every call returns 0 on success or a negative EC_ERR_* code; the message
 *    of the last failure on the calling thread is ec_last_error().  Nothing
 *    aborts, throws or exits across this boundary.  Asynchronous device
 *    faults surface at the next call that synchronises.
 *  - calls that take a hip stream (void*; NULL = the null stream) only
 *    enqueue work on it: no host synchronisation, no allocation.
 */
#ifndef EC_H_
#define EC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define EC_OK               0
#define EC_ERR_ARG         -1   /* invalid argument (null, size, range)     */
#define EC_ERR_DEVICE      -2   /* HIP runtime error                        */
#define EC_ERR_OOM         -3   /* device or host allocation failed         */
#define EC_ERR_UNSUPPORTED -4   /* valid but not implemented (N, d, kind)   */
#define EC_ERR_DOMAIN      -5   /* numerical precondition violated          */

/* ---- collision kernels -------------------------------------------------
 * B(g, w) = C_d |g|^gamma with C_2 = 1/(2 pi), C_3 = 1/(4 pi) (section 4.2).
 * In Carleman form (section 1, eq. Carleman)
 *   Bt(y, z) = 2^{d-1} C_d (|y|^2 + |z|^2)^{(gamma + 2 - d)/2},
 * which is constant (= 1/pi) -- hence separable in the fast algorithm --
 * for Maxwell molecules in 2D (gamma = 0) and hard spheres in 3D (gamma = 1).
 */
#define EC_KERNEL_MAXWELL     0   /* gamma = 0 (3D: non-separable)          */
#define EC_KERNEL_HARD_SPHERE 1   /* gamma = 1                              */
#define EC_KERNEL_VHS         2   /* 3D, -1 < gamma <= 1 (non-separable)    */
/*
 * Non-separable kernels (3D Maxwell, VHS): the fast algorithm needs products
 * alpha_{l+m} beta_l gamma_m (section 4.1); here the radius of y is
 * discretised by n_radial Gauss-Legendre nodes (rho_j, omega_j) on [0, R],
 * which separates the Carleman weight into M' = M n_radial products
 *   psi_{t,j}(k) = 2 omega_j rho_j cos(pi rho_j k.e_t / L),
 *   phi_{t,j}(k) = 4 pi int_0^R (rho_j^2 + r^2)^{(gamma-1)/2} J_0(q r) r dr,
 *                  q = pi |k_perp| / L (k_perp: the part of k orthogonal to e_t),
 * with the hard-sphere direction weights; gamma = 1 reproduces the
 * hard-sphere kernel as n_radial grows.
 */

/*
 * Truncation of the collision integral (the fast algorithm integrates the
 * Carleman form over a bounded set of (y, z)):
 *   EC_TRUNC_BOX:  |y| <= R and |z| <= R, the truncation of section 1.2 with
 *                  the box bound T >= (3 sqrt 2 + 1) R / 4;
 *   EC_TRUNC_BALL: |g| <= R in the classical form (eq. classical_hatB and the
 *                  remark after it; box bound T >= (3 + sqrt 2) R / 4).  With
 *                  y = (g + |g| w)/2, z = (g - |g| w)/2 (orthogonal,
 *                  |y|^2 + |z|^2 = |g|^2) this is the ball |y|^2 + |z|^2 <= R^2
 *                  of the same integrand: phi_{t,j} integrates over the disk of
 *                  radius sqrt(R^2 - rho_j^2), with rho_j = R sin(theta_j),
 *                  Gauss-Legendre in theta on [0, pi/2].  Non-separable (radial)
 *                  kernels only: 3D EC_KERNEL_MAXWELL and EC_KERNEL_VHS
 *                  (gamma = 1 gives hard spheres in this truncation).  3D
 *                  Maxwell with this truncation is the kernel of the paper's 3D
 *                  BKW experiment (section 4.2, Example 4, Table 3).
 */
#define EC_TRUNC_BOX  0
#define EC_TRUNC_BALL 1
/*
 * Angular factor of the classical form: B(g, w) = C_3 |g|^gamma b(cos theta),
 * cos theta = g.w / |g|, b(x) = sum_{i < n_bcos} bcos[i] x^i (n_bcos = 0:
 * b = 1, the isotropic kernels).  In the Carleman variables
 * cos theta = (|y|^2 - |z|^2) / (|y|^2 + |z|^2), a function of the two radii,
 * so it joins the radial weight of phi_{t,j} (3D radial kernels only, either
 * truncation).  b should be >= 0 on [-1, 1] for a physical kernel; the
 * library does not check it.
 */
#define EC_MAX_BCOS 8

typedef struct ec_kernel {
  int kind;          /* EC_KERNEL_*                                          */
  double gamma;      /* used by EC_KERNEL_VHS only                           */
  double R;          /* truncation radius of the Carleman integrals (section
                        1.2, eq. approximated_collision); R <= 0 selects the
                        largest R allowed by the truncation's box bound       */
  int n_radial;      /* radial nodes of a non-separable kernel (<= 0: 8)     */
  int unfiltered;    /* 0: the entropic method (Jackson filter sigma);
                        1: sigma = 1, the unfiltered Fourier collocation method
                        (eq. FCM) -- not positivity preserving; the comparison
                        of the positivity study (section 4.2, Fig. 2)        */
  int truncation;    /* EC_TRUNC_BOX (0) or EC_TRUNC_BALL (1)                 */
  int n_bcos;        /* 0 .. EC_MAX_BCOS coefficients of b(cos theta)        */
  double bcos[EC_MAX_BCOS];   /* b(x) = sum_i bcos[i] x^i (copied by the
                                  plan; unused entries ignored)              */
} ec_kernel;

/* ---- precision of the transforms --------------------------------------- */
#define EC_FP64   0   /* transforms, products and sums in FP64              */
#define EC_FP32   1   /* transforms and products in FP32, sum over terms,
                         loss combine and reductions in FP64                */
#define EC_BF16X3 2   /* as EC_FP32, but the inverse DFT along x of every term
                         runs on MFMA as a real (2N x 2N) DFT-matrix product
                         with split-BF16 operands (hi*hi + hi*lo + lo*hi, FP32
                         accumulate); 3D cells with N = 16, 32 or 64 only    */

typedef struct ec_plan ec_plan;
typedef struct ec_batch ec_batch;

/*
 * ec_setup_kernel -- build the tables of one (N, d, L, kernel, M) on the
 * current HIP device: the quadrature rules, the filter and the radial fits
 * are computed on the host, the per-mode multipliers (FP64, plus an FP32 copy
 * for plans that allow FP32 batches) by a kernel on the device; the call
 * synchronizes the device before it returns.
 *   N      points per axis; supported: d = 3: 8, 12, 16, 24, 32, 64, 128
 *          (128: FP64 only, lines schedule); d = 2: 8, 12, 16, 24, 32, 64, 128,
 *          256, 512 (N >= 64: FP64 only).
 *   d      2 or 3.
 *   L      half-width of the velocity box (> 0).
 *   M      number of products in the gain: d = 2: samples theta_t = t pi/(2M)
 *          in [0, pi/2), each paired with theta_t + pi/2 (section 4.1, eq.
 *          discrete_hatB; section 4.2, Table 2 convention); d = 3: directions
 *          of a hemisphere product rule (Gauss-Legendre in cos(theta) times
 *          uniform azimuth, positive weights summing to 2 pi).
 * Precomputes (section 3.2.2, eq. JacksonFilter2; section 4.1):
 *   sigma(k)  the modified Jackson filter, n = N/2 for even N (sigma(-N/2) = 0);
 *   alpha_t(k) = N^-d w_t sigma(k) psi_t(k),  beta_t(k) = N^-d sigma(k) phi_t(k),
 *   D(k) = N^-d sigma(k)^2 sum_t w_t psi_t(k) phi_t(k)  (the diagonal
 *   B^s(k,k) of the same low-rank kernel, which gives exact mass conservation).
 * The plan owns its device memory until ec_plan_destroy.
 */
int ec_setup_kernel(int N, int d, double L, const ec_kernel* kernel, int M,
                    ec_plan** out);
int ec_plan_destroy(ec_plan* plan);

/* Number of gain products M' of the plan (M for the separable kernels,
 * M n_radial for the non-separable ones). */
int ec_plan_terms(const ec_plan* plan, int* n_terms);

/*
 * ec_plan_tables -- host copy of the plan's FP64 device tables, for
 * inspection (a synchronous device-to-host copy).
 * gamma: [M'+1][N^d] complex numbers stored as (re, im) FP64 pairs, modes in
 * FFT index order (index i holds the mode i for i < N/2, i - N otherwise),
 * axes ordered (k0, k2, k1) -- first axis slowest, then the last axis, then
 * the middle axis fastest (d = 2: (k1_is_absent) i.e. [k_last][k_first]).
 * Entry t < M' is alpha_t + i beta_t; entry M' is D + 0 i.
 * Host memory owned by the caller; size = 2 (M'+1) N^d doubles.
 */
int ec_plan_tables(const ec_plan* plan, double* gamma);

/* Same tables without a device (host only; used by CPU tests). */
int ec_host_tables(int N, int d, double L, const ec_kernel* kernel, int M,
                   int* n_terms, double* gamma /* may be NULL to query */);

/*
 * ec_host_table_modes -- the same table entries at a list of modes only
 * (host only), for checking plans whose full tables are large.
 *   modes: [n_modes] flat mode indices in the table layout of
 *   ec_plan_tables, idx = (k0 N + k2) N + k1 (d = 2: k2 N + k1), each in
 *   [0, N^d); out of range -> EC_ERR_ARG.
 *   gamma: [M'+1][n_modes] complex (re, im) FP64 pairs, caller-owned,
 *   2 (M'+1) n_modes doubles; may be NULL to query n_terms.
 */
int ec_host_table_modes(int N, int d, double L, const ec_kernel* kernel, int M,
                        int64_t n_modes, const int64_t* modes, int* n_terms,
                        double* gamma);

/*
 * ec_batch_create -- a packed batch of cells grouped by plan.
 *   plans[g], counts[g]: group g holds counts[g] cells of plans[g] (the plans
 *   must stay alive while the batch exists).
 *   precision: EC_FP64, EC_FP32 or EC_BF16X3.
 * Layout of f and Q for every call on the batch: cells in group order, each
 * cell N_g^d contiguous FP64 values starting at a 256-byte aligned element
 * offset (ec_batch_offsets).  Workspaces for all later calls are allocated
 * here; ec_collide and ec_step never allocate.
 */
int ec_batch_create(const ec_plan* const* plans, const int64_t* counts,
                    int n_groups, int precision, ec_batch** out);
int ec_batch_destroy(ec_batch* batch);
/* n_cells; total FP64 elements of the packed array (including padding). */
int ec_batch_size(const ec_batch* batch, int64_t* n_cells, int64_t* n_elems);
/* offsets[c] = element offset of cell c (host array of n_cells). */
int ec_batch_offsets(const ec_batch* batch, int64_t* offsets);
/*
 * Execution schedule of the 3D groups (2D groups always use the two-pass
 * schedule).  EC_SCHED_PIPELINE: one software-pipelined launch per chunk of
 * cells_per_pass cells, whose four roles (forward transform, x pass, slab
 * pass split into term_groups groups of terms, combine) work on four
 * consecutive chunks, so the per-term intermediates of a chunk stay in the
 * last-level cache.  EC_SCHED_TWO_PASS: three launches per chunk with the
 * intermediates of the whole chunk in memory.  EC_SCHED_FUSED (3D, N = 16,
 * 24, 32; FP64 and FP32): forward transform, then one kernel that runs every
 * term's inverse transform on chip (the x axis split by decimation in
 * frequency into term_groups residue classes, one workgroup per class) and
 * accumulates the gain in FP64 registers, so no per-term intermediate touches
 * device memory; splits: N = 16: 1, 2; N = 24: 2, 3; N = 32: 2, 4 (at 32^3
 * the term volume is held in registers, one column or line per thread).
 * EC_SCHED_LINES (3D, N = 64, 128; FP64): every axis by line FFTs in LDS,
 * one term at a time through device memory (per cell of a pass: spectrum and
 * term volume, complex FP64, and an FP64 accumulator, 40 N^3 bytes); the only
 * schedule of 128^3 grids, whose plans are FP64 only.  EC_SCHED_TERMS (3D,
 * N = 16, 24, 32; FP64 and FP32; the fused schedule's splits, default 4 at
 * 32^3): the fused schedule's kernel run with one workgroup per (cell,
 * term, residue class), each writing its
 * term's products to device memory (J N^3 FP64 values per cell of a pass),
 * then a kernel that sums them per point in the fused kernel's order; for
 * small batches, whose latency is then about one term's.
 * 0 for cells_per_pass or term_groups selects the default (chosen from the
 * cache size); the autotuner picks measured values.  A new batch starts 3D
 * groups on the term-parallel schedule up to its measured crossover with the
 * fused one (FP64 / FP32: N = 16 192 / 192 cells, N = 24 64 / 80, N = 32
 * 48 / 40), larger groups on the fused schedule where it exists (default
 * split by cells per launch: 4 at 32^3 up to a quarter of the CU count,
 * 2 at 24^3 where two workgroups per cell fill one round over the CUs and
 * three do not, else 1 at 16^3, 3 at 24^3 and 2 at 32^3), other 3D
 * groups of N <= 32 below 32 cells on the pipelined schedule, and the rest
 * on the two-pass schedule.
 * Reallocates the workspace (synchronises the device); call it outside
 * graph capture.
 */
#define EC_SCHED_PIPELINE 0
#define EC_SCHED_TWO_PASS 1
#define EC_SCHED_FUSED 2
#define EC_SCHED_LINES 3
#define EC_SCHED_TERMS 4
int ec_batch_set_schedule(ec_batch* batch, int group, int mode, int cells_per_pass,
                          int term_groups);
int ec_batch_get_schedule(const ec_batch* batch, int group, int* mode, int* cells_per_pass,
                          int* term_groups);
/*
 * ec_autotune -- measure candidate schedules of every group on the device
 * (two-pass with several chunk sizes; for 3D also the pipelined schedule over
 * chunk sizes and term groups), keep the fastest, and append it to the text
 * cache at cache_path (one line per key "arch|d|N|M|kind|L|R|precision|cells";
 * NULL or "" = no cache).  A cached key is applied without measuring unless
 * flags has EC_TUNE_REMEASURE.  f should hold representative cells; Q is
 * overwritten.  Synchronises the stream; not capturable.
 */
#define EC_TUNE_REMEASURE 1
int ec_autotune(ec_batch* batch, const double* f, double* Q, const char* cache_path, int flags,
                void* hip_stream);

/* Shorthand: change only cells_per_pass of a group. */
int ec_batch_set_chunk(ec_batch* batch, int group, int cells_per_pass);

/*
 * ec_collide -- Q = Q^s[F] for every cell of the batch (section 3.2.2, eq. Qsr
 * evaluated by the fast algorithm of section 4.1).  f, Q: device arrays of
 * ec_batch_size().n_elems FP64; f and Q must not alias.  Padding is ignored.
 */
int ec_collide(ec_batch* batch, const double* f, double* Q, void* hip_stream);

/*
 * ec_collide_noalloc -- ec_collide without any device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Q^s of n_cells contiguous 3D
 * cells of `plan` (N = 16, 24 or 32; f and Q each hold n_cells x N^3 FP64
 * values, cell c at offset c N^3, C order [x][y][z]; device memory owned by
 * the caller, not aliased), on the fused schedule of ec_collide (same
 * kernels, same x split for the same cells per launch) in precision EC_FP64
 * or EC_FP32.  Its only device memory beyond f and Q is a fixed scratch
 * array of EC_NOALLOC_SCRATCH_BYTES that the library's code object holds on
 * every device it runs on until the process ends (the half-space spectra of
 * one pass of cells and their offsets: 255 cells of 32^3 in FP64 per pass;
 * more cells run in passes).  Every call on a device shares that device's
 * scratch: calls that overlap on one device (other streams, other threads)
 * race and must be ordered by the caller.  Nothing in the scratch needs
 * clearing between calls.  Stream-ordered on hip_stream, no host sync.
 * Errors: EC_ERR_ARG (null or aliased pointers, n_cells < 0, a precision
 * other than EC_FP64/EC_FP32, a plan of another device), EC_ERR_UNSUPPORTED
 * (a plan other than 3D N = 16, 24, 32, or one cell larger than the
 * scratch), EC_ERR_DEVICE (launch failure).
 */
#define EC_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int ec_collide_noalloc(const ec_plan* plan, int precision, int64_t n_cells, const double* f,
                       double* Q, void* hip_stream);

/*
 * ec_entropy_prod -- per cell, out[c] = h^d sum_{F_r > 0} Q_r ln F_r (the
 * discrete H-functional of Theorem 1, eq. Htheorem; <= 0 in exact arithmetic
 * for F >= 0) and, if n_nonpos != NULL, n_nonpos[c] = #{r : F_r <= 0}.
 * Deterministic (fixed reduction order).  Device arrays.
 */
int ec_entropy_prod(ec_batch* batch, const double* f, const double* Q,
                    double* out, int32_t* n_nonpos, void* hip_stream);

/*
 * ec_monitors -- per cell EC_NMON FP64 diagnostics of (f, Q), device array
 * out[c * EC_NMON + i]: mass h^d sum F, sum Q, h^d sum_{F>0} Q ln F,
 * eta = h^d sum_{F>0} F ln F (section 4.2), min F, the positivity error
 * epsilon = (sum|F| - sum F)/sum|F| (section 4.2), sum |Q|, the momentum
 * h^d sum Q v (three components; the third is 0 in 2D) and the energy
 * h^d sum Q |v|^2 of Q at the grid points v = -L + j h.  Only mass is
 * conserved exactly by the method; momentum and energy are reported, not
 * conserved (section 5).
 */
#define EC_NMON 11
#define EC_MON_MASS      0
#define EC_MON_SUMQ      1
#define EC_MON_ENTPROD   2
#define EC_MON_ETA       3
#define EC_MON_MINF      4
#define EC_MON_EPS       5
#define EC_MON_SUMABSQ   6
#define EC_MON_MOMQ      7   /* 7, 8, 9: h^d sum Q v_i */
#define EC_MON_ENERGYQ  10
int ec_monitors(ec_batch* batch, const double* f, const double* Q, double* out,
                void* hip_stream);

/*
 * ec_step_graph -- n_steps forward-Euler steps F <- F + dt Q^s[F] of the EFM
 * ODE (section 3.3, eq. modifiedIVP), in place on f.  The steps are captured
 * into one HIP graph (every step's kernels and monitors as graph nodes, up to
 * 200 steps per graph; a longer run launches that graph repeatedly and a
 * second graph for the remainder) and launched on hip_stream; the graphs are
 * kept and reused while (f, dt, monitors, n_steps) stay the same.  The first
 * call for new arguments captures and instantiates (no device allocation);
 * later calls only launch.  If monitors != NULL it receives, per step and
 * cell, (mass, eta) of the state after the step:
 * monitors[(s * n_cells + c) * 2 + i], device memory of n_steps * n_cells * 2
 * doubles owned by the caller.  Positivity is kept when dt max_r l_r <= 1
 * (proof of Theorem 1).  Errors: EC_ERR_ARG for dt <= 0 or n_steps < 0.
 * ec_step is the same call under its earlier name.
 */
int ec_step_graph(ec_batch* batch, double* f, double dt, int n_steps,
                  double* monitors, void* hip_stream);
int ec_step(ec_batch* batch, double* f, double dt, int n_steps,
            double* monitors, void* hip_stream);

/*
 * ec_step_ssprk3 -- n_steps steps of the third-order strong-stability-
 * preserving Runge-Kutta method (the time integrator of the paper's numerical
 * experiments, section 4; Shu-Osher form: u1 = f + dt Q(f), u2 = 3/4 f +
 * 1/4 (u1 + dt Q(u1)), f <- 1/3 f + 2/3 (u2 + dt Q(u2))), in place on f,
 * with the same graphs, monitors and arguments as ec_step_graph.  Each step
 * is a convex combination of forward-Euler steps, so the positivity condition
 * of ec_step applies per stage.  The first call allocates two stage buffers
 * of the batch's size (synchronises the device; call it outside capture).
 */
int ec_step_ssprk3(ec_batch* batch, double* f, double dt, int n_steps, double* monitors,
                   void* hip_stream);

/*
 * Profiling of ec_collide (tracing).  While enabled, ec_collide records HIP
 * events on its stream around its kernels.  ec_profile_read waits for them and
 * returns, per group g of the batch and kernel k (EC_PROF_KERNELS per group:
 * 0 forward transform (the slab transform of the two-pass schedule, the
 * whole 3D transform of the fused and term-parallel schedules; 2D cells run
 * as one block each include it in 5), 1 x-pencil
 * pass, 2 slab pass of the two-pass schedule, 3 the pipelined kernel, 4
 * reserved (always 0), 5 fused or term-parallel kernels), ms[6g + k] = summed
 * duration and launches[6g + k] = number of launches, and cells[g] = cells
 * processed; then it forgets the records.  Host arrays of 6 * n_groups
 * (cells: n_groups).
 */
#define EC_PROF_KERNELS 6
int ec_profile(ec_batch* batch, int enable);
int ec_profile_read(ec_batch* batch, double* ms, int64_t* launches, int64_t* cells);

/*
 * ec_copy -- dst[i] = src[i], i < n, with a plain grid-stride copy kernel
 * (k_copy).  Used to calibrate hardware byte counters: its algorithmic
 * traffic is exactly 16 n bytes.  Device arrays, must not overlap.
 */
int ec_copy(const double* src, double* dst, int64_t n, void* hip_stream);

/*
 * ec_valu_probe -- measured vector-ALU throughput of the current device, for
 * rooflines against the device as it runs: 8192 blocks x 256 threads, each
 * with 16 independent fused multiply-add chains of 2048 steps (2 flops per
 * step), two warm-up launches, then the fastest of five launches timed with
 * HIP events on hip_stream; the call synchronizes on them.  precision: EC_FP64 or
 * EC_FP32 (FP32 arithmetic is unpacked in this library, so its rate is not
 * the packed-FP32 peak).  *tflops receives TFLOP/s.  Allocates and frees 8
 * bytes of device memory.
 */
int ec_valu_probe(int precision, double* tflops, void* hip_stream);

/* ---- learned surrogate ---------------------------------------------------
 * A Fourier neural operator that predicts c0^2 Q / mass^2 from c0 F / mass
 * on the N^3 grid (Q is quadratic in F; c0 = (2 pi)^{3/2} puts the peak of a
 * unit-temperature Maxwellian at 1): lift 1 -> C channels, `layers` layers
 * u <- GELU(W u + b + S(u)) (no GELU after the last), projection C -> 1;
 * S keeps the modes kx, ky in [-modes, modes), kz in [0, modes) with complex
 * C x C weights per mode, between a forward DFT and a normalised (1/n)
 * inverse DFT.  FP32 parameters, trained by the library's own
 * forward, backward and Adam kernels on (F, Q) pairs of the exact operator.
 * Supported (N, modes, channels): (32, 12, 16), (16, 6, 8), (8, 2, 4).
 */
typedef struct ec_surrogate ec_surrogate;
int ec_surrogate_create(int N, int modes, int channels, int layers, uint64_t seed, int max_batch,
                        ec_surrogate** out);
int ec_surrogate_destroy(ec_surrogate* s);
int ec_surrogate_num_params(const ec_surrogate* s, int64_t* n);
/* Host copies of the flat FP32 parameter / last-gradient vector (num_params
 * floats; layout: Wl[C], bl[C], then per layer W[C][C], b[C], R[modes][C][C]
 * as (re, im) pairs, then Wp[C], bp).  set_params resets the Adam state. */
int ec_surrogate_get_params(const ec_surrogate* s, float* host);
int ec_surrogate_set_params(ec_surrogate* s, const float* host);
int ec_surrogate_get_grads(const ec_surrogate* s, float* host);
/* Normalised training inputs of cells cell0 .. cell0+B-1 of a batch (one
 * group of 3D cells of the surrogate's N): Fin = c0 F / mass and, if Q and
 * target are not NULL, target = c0^2 Q / mass^2 (device [B][N^3] FP32). */
int ec_surrogate_prepare(ec_surrogate* s, const ec_batch* batch, const double* f, const double* Q,
                         int64_t cell0, int B, float* Fin, float* target, void* hip_stream);
/* y = network(Fin), device [B][N^3] FP32, B <= max_batch. */
int ec_surrogate_forward(ec_surrogate* s, const float* Fin, float* y, int B, void* hip_stream);
/* One forward + backward (per-sample relative squared error, averaged) and,
 * if update != 0, one Adam step (lr, beta 0.9/0.999).  If loss != NULL the
 * mean loss is returned (synchronises the stream). */
int ec_surrogate_train(ec_surrogate* s, const float* Fin, const float* target, int B,
                       float lr, int update, double* loss, void* hip_stream);
/* The same call under its earlier name. */
int ec_surrogate_train_step(ec_surrogate* s, const float* Fin, const float* target, int B,
                            float lr, int update, double* loss, void* hip_stream);
/* Screened inference on a batch (one group of 3D cells of the surrogate's N):
 * Q = mass^2 network(c0 F / mass) / c0^2, then projected orthogonally onto
 * zero discrete mass (Q - mean Q; the exact operator conserves mass exactly,
 * so the projection cannot move Q farther from it in the 2-norm).  A cell
 * passes the
 * screen when the discrete H-functional of the projected Q,
 * h^3 sum_{F>0} Q ln F, is <= 0 (Theorem 1), and the raw prediction's
 * residuals |sum Q| <= tau_m sum |Q|, |sum Q v| / (L sum|Q|) <= tau_e and
 * |sum Q |v|^2| / (3 L^2 sum|Q|) <= tau_e.  Every failing cell is
 * recomputed with the exact operator (ec_collide on a compacted batch).
 * tau_e < 0 skips the momentum and energy checks (the library's default
 * screen, tau_m = 5e-3 and tau_e < 0: on held-out cells it accepts ~97 %
 * with a largest relative L2 error of 3.2 %, inside the stated 5e-2).
 * tau_m < 0 disables the screen: every cell keeps the projected prediction
 * (the screen values are still written).
 * Optional device outputs: fell_back[c] (0/1), screen[c*4 + {P, mass, mom,
 * energy residual}]; host output n_fallback.  Synchronises the stream. */
int ec_surrogate_collide(ec_surrogate* s, ec_batch* batch, const double* f, double* Q,
                         double tau_m, double tau_e, int32_t* fell_back, double* screen,
                         int64_t* n_fallback, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* ec_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EC_H_ */

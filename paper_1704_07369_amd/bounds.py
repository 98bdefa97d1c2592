"""Stated error bounds of the reduced-precision paths, fixed a priori from the
arithmetic (not fitted to measurements).

Metric (the same for every path): ||Q - Q_ref||_2 / ||Q+_ref||_2 over one
cell's grid, Q+ the gain (Q itself nearly vanishes near equilibrium while
the transform rounding scales with the gain).

FP64 path: 1e-12.

FP32 transforms, FP64 sums (EC_FP32).  Each term w_t a_t b_t of the gain
needs two length-n transforms of a spectrum held in FP32 (n = N^d): the
forward transform of F, the multiply by the FP32 table, and the inverse
transform.  For a radix-2/4 FFT in precision u the computed transform
satisfies ||X^ - X||_2 <= log2(n) eta ||X||_2 to first order, with
eta = mu + gamma_4 (sqrt 2 + mu) ~ (4 sqrt 2 + 1) u and mu ~ u the error of
the stored twiddles (Higham, Accuracy and Stability of Numerical
Algorithms, 2nd ed., Thm. 24.2).  Splitting one axis by decimation in
frequency changes how the stages are grouped, not the length, so log2(n)
stays.  The FP32 spectrum, the FP32 table entry and the FP32 product add
3 u.  Each of a_t, b_t thus carries a normwise relative error of at most
    e1 = 2 log2(n) (4 sqrt 2 + 1) u + 3 u,     u = 2^-24,
and a_t b_t at most 2 e1 relative to |a_t| |b_t|.  For non-negative F the
a_t, b_t are non-negative (smoothed line and disk integrals of F, the
positivity argument of section 4.1) and the weights are positive, so
sum_t w_t |a_t b_t| = Q+ and the gain's error is at most 2 e1 ||Q+||.  The
loss Q- = F l takes one transform of the same length (l carries e1, F is
exact), adding e1 ||Q-||.  So
    ||dQ||_2 / ||Q+||_2 <= e1 (2 + r),   r = ||Q-||_2 / ||Q+||_2,
fp32_bound(N, d, r).  e1 at 16^3: 9.7e-6, 24^3: 1.11e-5, 32^3: 1.21e-5,
64^3: 1.45e-5, 2D 32^2: 8.1e-6 (with r = 1: 2.4e-5 .. 4.3e-5).  Every
schedule (two-pass, fused, term-parallel) performs transforms of these
lengths, so one bound serves all of them.

Split-BF16 x pass (EC_BF16X3): the x pass of every inverse transform is a
length-N DFT written as a real GEMM with both operands split x = hi + lo
(hi = bf16(x), lo = bf16(x - hi): |x - hi - lo| <= 2^-16 |x|, bf16 has an
8-bit significand), the product lo*lo dropped (<= 2^-16 |w||x|), FP32
accumulation.  Each term of the matrix-vector product is off by at most
3 * 2^-16 |w||x|; with |W_jk| = 1, || |W||x| ||_2 <= N ||x||_2 while
||W x||_2 = sqrt(N) ||x||_2, so the pass adds 3 * 2^-16 sqrt(N) to e1:
    bf16x3_bound(N, d, r) = (e1 + 3 * 2^-16 sqrt(N)) (2 + r).
With r = 1: 16^3 5.8e-4, 32^3 8.1e-4, 64^3 1.1e-3.

These are worst-case first-order bounds; independent rounding errors mostly
cancel, so measured errors sit one to two orders of magnitude below them.
"""
from __future__ import annotations

import math

U32 = 2.0 ** -24
FP64_BOUND = 1e-12


def e1_fp32(N: int, d: int) -> float:
    """Normwise relative error of one FP32 forward + inverse transform pair."""
    return 2.0 * math.log2(N ** d) * (4.0 * math.sqrt(2.0) + 1.0) * U32 + 3.0 * U32


def fp32_bound(N: int, d: int, loss_ratio: float = 1.0) -> float:
    return e1_fp32(N, d) * (2.0 + loss_ratio)


def bf16x3_bound(N: int, d: int, loss_ratio: float = 1.0) -> float:
    return (e1_fp32(N, d) + 3.0 * 2.0 ** -16 * math.sqrt(N)) * (2.0 + loss_ratio)


def bound(precision: int, N: int, d: int, loss_ratio: float = 1.0) -> float:
    """precision: 0 FP64, 1 FP32, 2 split-BF16 (the EC_* codes); loss_ratio
    = ||Q-||_2 / ||Q+||_2 of the reference."""
    if precision == 0:
        return FP64_BOUND
    if precision == 1:
        return fp32_bound(N, d, loss_ratio)
    if precision == 2:
        return bf16x3_bound(N, d, loss_ratio)
    raise ValueError(f"precision {precision}")

"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the collision operator.  It only fixes the
velocity grid convention of the input contract (point samples on a uniform grid,
section 2 "Initial condition", eq. I_N) and draws the parameters of the test
distributions from a seeded PCG64 generator.

Grid convention: the box is [-L, L]^d, the step is h = 2L/N and the j-th sample
along an axis sits at v_j = -L + j*h, j = 0..N-1 (section 1.1, eq. X, shifted to
start at the left edge; the operator is translation-equivariant so the offset
does not change the method).  Arrays are C-ordered with the last axis fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "grid_1d", "velocity_grid", "Gaussian", "Mixture", "mixture_two_gaussians",
    "mixture_anisotropic", "sample_mixture", "bkw", "bkw_datum",
    "batch_mixed_sizes", "rng", "trig_polynomial",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def grid_1d(N: int, L: float) -> np.ndarray:
    h = 2.0 * L / N
    return -L + h * np.arange(N, dtype=np.float64)


def velocity_grid(N: int, d: int, L: float):
    """Return the d coordinate arrays (each of shape (N,)*d) of the grid."""
    v = grid_1d(N, L)
    return np.meshgrid(*([v] * d), indexing="ij")


@dataclass
class Gaussian:
    weight: float
    mean: np.ndarray          # (d,)
    temp: np.ndarray          # (d,) diagonal temperatures


@dataclass
class Mixture:
    d: int
    comps: list = field(default_factory=list)


def mixture_two_gaussians(seed: int, d: int, mean_box: float = 2.0,
                          t_lo: float = 0.5, t_hi: float = 1.5) -> Mixture:
    """Two isotropic Gaussians: centres U[-2,2]^d, temperatures U[t_lo,t_hi],
    weights (w, 1-w) with w ~ U(0,1).  Generalises the bi-Gaussian datum of
    section 4.2 (Example 2)."""
    g = rng(seed)
    w = float(g.uniform(0.0, 1.0))
    comps = []
    for wk in (w, 1.0 - w):
        mu = g.uniform(-mean_box, mean_box, size=d)
        t = float(g.uniform(t_lo, t_hi))
        comps.append(Gaussian(wk, mu, np.full(d, t)))
    return Mixture(d, comps)


def mixture_anisotropic(seed: int, d: int, kmin: int = 2, kmax: int = 4,
                        mean_box: float = 2.0, t_lo: float = 0.3,
                        t_hi: float = 2.0) -> Mixture:
    """K ~ U{kmin..kmax} anisotropic Gaussians with means U[-2,2]^d, diagonal
    temperatures U[t_lo, t_hi] and Dirichlet(1,...,1) weights."""
    g = rng(seed)
    K = int(g.integers(kmin, kmax + 1))
    w = g.dirichlet(np.ones(K))
    comps = []
    for k in range(K):
        mu = g.uniform(-mean_box, mean_box, size=d)
        t = g.uniform(t_lo, t_hi, size=d)
        comps.append(Gaussian(float(w[k]), mu, t))
    return Mixture(d, comps)


def sample_mixture(mix: Mixture, N: int, L: float) -> np.ndarray:
    """Point samples F_r = f(v_r) of the mixture on the N^d grid (FP64)."""
    V = velocity_grid(N, mix.d, L)
    F = np.zeros(V[0].shape, dtype=np.float64)
    for c in mix.comps:
        e = np.zeros_like(F)
        norm = 1.0
        for i in range(mix.d):
            e += (V[i] - c.mean[i]) ** 2 / (2.0 * c.temp[i])
            norm *= 1.0 / math.sqrt(2.0 * math.pi * c.temp[i])
        F += c.weight * norm * np.exp(-e)
    return F


def bkw(d: int, t: float, N: int, L: float) -> np.ndarray:
    """Samples of the BKW solution for Maxwell molecules (section 4.2,
    Example 1 for d=2 and Example 4 for d=3) at time t."""
    V = velocity_grid(N, d, L)
    v2 = sum(x * x for x in V)
    if d == 2:
        S = 1.0 - math.exp(-t / 8.0) / 2.0
        return (1.0 / (2.0 * math.pi * S) * np.exp(-v2 / (2.0 * S))
                * ((2.0 * S - 1.0) / S + (1.0 - S) / (2.0 * S * S) * v2))
    if d == 3:
        S = 1.0 - 2.0 * math.exp(-t / 6.0) / 5.0
        return ((2.0 * math.pi * S) ** -1.5 * np.exp(-v2 / (2.0 * S))
                * ((5.0 * S - 3.0) / (2.0 * S) + (1.0 - S) / (2.0 * S * S) * v2))
    raise ValueError("d must be 2 or 3")


def bkw_datum(d: int, N: int, L: float) -> np.ndarray:
    return bkw(d, 0.0, N, L)


def batch_mixed_sizes(seed: int, n_cells: int, sizes=(16, 24, 32),
                      fractions=(0.40, 0.35, 0.25)) -> np.ndarray:
    """Grid size of each cell of a mixed batch: exact counts from the
    fractions (remainder to the first size), shuffled by a seeded permutation."""
    counts = [int(round(f * n_cells)) for f in fractions]
    counts[0] += n_cells - sum(counts)
    arr = np.concatenate([np.full(c, s, dtype=np.int64) for s, c in zip(sizes, counts)])
    return rng(seed).permutation(arr)


def trig_polynomial(seed: int, N: int, d: int, L: float, n_waves: int = 12,
                    kmax: int | None = None, background: float = 1.0):
    """A real trigonometric polynomial on the grid with a known, small set of
    frequencies: F(v) = background + sum over n_waves random integer vectors
    k (components in [-kmax, kmax], distinct, k != 0) of
    2 Re(c_k exp(i pi k.v / L)), c_k complex with |c_k| <= 1/(4 n_waves), so
    F stays within background +- 1/2.  Returns (F, modes): modes is the
    (d, 2 n_waves + 1) integer array of the frequencies present (0, the k and
    their negatives).  For parity tests of large plans, whose reference
    needs the kernel factors only on these modes."""
    g = rng(seed)
    kmax = N // 2 - 2 if kmax is None else kmax
    chosen = set()
    while len(chosen) < n_waves:
        k = tuple(int(x) for x in g.integers(-kmax, kmax + 1, d))
        if any(k) and k not in chosen and tuple(-x for x in k) not in chosen:
            chosen.add(k)
    ks = np.array(sorted(chosen), dtype=np.int64)                 # (n_waves, d)
    amp = g.uniform(0.0, 1.0 / (4 * n_waves), n_waves)
    ph = g.uniform(0.0, 2.0 * math.pi, n_waves)
    v = velocity_grid(N, d, L)
    F = np.full((N,) * d, float(background))
    for k, a, p in zip(ks, amp, ph):
        arg = sum(math.pi / L * kk * vv for kk, vv in zip(k, v))
        F += 2.0 * a * np.cos(arg + p)
    modes = np.concatenate([np.zeros((1, d), np.int64), ks, -ks]).T
    return F, modes


"""FP64 CPU oracle of the entropic Fourier method (EFM) collision operator.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of bench.py may import this module.  It shares no code with the HIP
library: every table here is computed from the defining integrals by
quadrature (the library uses closed forms), every transform is a library FFT
or an explicit exponential sum, and the collision term is the plain double
sum of the paper.

What it computes (citations are to the paper, arXiv 1704.07369):

* grid X and mode set K (section 1.1, eq. X; section 1.2, eq. K), the DFT pair
  (section 2, eq. DFT) and the trigonometric basis E_k(v) = exp(i pi k.v / T);
* the modified Jackson filter (section 3.2.2, eq. JacksonFilter2) and its
  tensor product;
* the low-rank kernel modes of the fast algorithm (section 4.1, eq. fastAlg,
  eq. spherical_hatB, eq. fast_hatB, eq. discrete_hatB) -- in 2D literally,
  in 3D by the same polar decomposition carried one dimension up;
* the entropic collision term in Fourier space (section 3.2.2, eq. Qsk), by
  the O(T n^2) double sum (C code in csrc/efm_direct.c), and back on the grid
  (eq. Qsr);
* the same quantity evaluated point by point through the factorised fast
  algorithm with explicit exponential sums (section 3.1.1, eq. fastFGM, with
  the collocation evaluation of eq. FGM_Qcv) -- for large grids;
* the DVM coefficients A^sigma (section 3.2, eq. A_simplified with the
  filtered kernel, eq. tildetildeA) and the DVM form of Q (eq. Qsr), brute
  force on tiny grids;
* diagnostics: mass, entropy (section 4.2, eta), positivity error epsilon,
  the discrete H-functional of Theorem 1;
* forward Euler and the SSP-RK3 step (section 4.1), BKW closed forms.

Readings of the paper (fixed by reproducing Table 2 to every printed digit, or
chosen where the paper is silent), in short:
the even-N filter is eq. JacksonFilter2 evaluated with n = N/2; the 2D nodes
are theta_t = t*pi/(2M), t = 0..2M-1; the 3D nodes are a hemisphere product
rule (Gauss-Legendre in cos(theta) folded onto [0,1], uniform azimuth).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_efm_direct.so")
_lib = None

KIND_MAXWELL = "maxwell"          # B = C_d |g|^0
KIND_HARD_SPHERE = "hard_sphere"  # B = C_d |g|^1
KIND_VHS = "vhs"                  # B = C_d |g|^gamma (3D Maxwell is gamma = 0)

# Section 4.2: B(g, w) = 1/(2 pi) in 2D and 1/(4 pi) in 3D for Maxwell
# molecules; the hard-sphere kernel keeps the same constant times |g|.
C_D = {2: 1.0 / (2.0 * math.pi), 3: 1.0 / (4.0 * math.pi)}


def default_box(R: float) -> float:
    """Smallest half-width with T >= (3 sqrt 2 + 1) R / 4 (section 1.2)."""
    return (3.0 * math.sqrt(2.0) + 1.0) * R / 4.0


def classical_box(R: float) -> float:
    """Smallest half-width with T >= (3 + sqrt 2) R / 4, the bound of the
    remark on the classical form (section 1.2, eq. classical_hatB)."""
    return (3.0 + math.sqrt(2.0)) * R / 4.0


# ----------------------------------------------------------------------------
# Grid, modes, DFT
# ----------------------------------------------------------------------------

def modes_1d(N: int) -> np.ndarray:
    """Mode values in FFT index order: 0..ceil(N/2)-1, -floor(N/2)..-1."""
    return np.fft.fftfreq(N, d=1.0 / N).round().astype(np.int64)


def mode_grid(N: int, d: int):
    k = modes_1d(N)
    return [x.ravel() for x in np.meshgrid(*([k] * d), indexing="ij")]


def grid_points(N: int, d: int, L: float):
    v = -L + (2.0 * L / N) * np.arange(N)
    return [x.ravel() for x in np.meshgrid(*([v] * d), indexing="ij")]


def E(k_list, v_list, L):
    """E_k(v) = exp(i pi k.v / L) for all pairs (rows: points v, cols: modes k)."""
    ph = np.zeros((len(v_list[0]), len(k_list[0])))
    for kd, vd in zip(k_list, v_list):
        ph += np.outer(vd, kd)
    return np.exp(1j * math.pi / L * ph)


def dft(F: np.ndarray, L: float) -> np.ndarray:
    """Fh_k = N^-d sum_p F_p E_{-k}(p) (section 2, eq. DFT) on the grid
    v_j = -L + j h.  Uses a library FFT as the summation step; the left-edge
    offset of the grid contributes the explicit phase exp(i pi sum k)."""
    d = F.ndim
    N = F.shape[0]
    ks = np.meshgrid(*([modes_1d(N)] * d), indexing="ij")
    phase = np.exp(1j * math.pi * sum(ks))
    return phase * np.fft.fftn(F) / N ** d


def idft(Fh: np.ndarray, L: float) -> np.ndarray:
    """F_p = sum_k Fh_k E_k(p) (section 2, eq. DFT)."""
    d = Fh.ndim
    N = Fh.shape[0]
    ks = np.meshgrid(*([modes_1d(N)] * d), indexing="ij")
    phase = np.exp(-1j * math.pi * sum(ks))
    return np.fft.ifftn(phase * Fh) * N ** d


# ----------------------------------------------------------------------------
# Modified Jackson filter (section 3.2.2, eq. JacksonFilter2)
# ----------------------------------------------------------------------------

def jackson_n(N: int) -> int:
    """The n of eq. JacksonFilter2: (N-1)/2 for odd N (the paper's N = 2n+1);
    for even N the reading that reproduces Table 2 is n = N/2, so that the
    mode -N/2 gets sigma = 0 (section 4.1, even-N remark)."""
    return (N - 1) // 2 if N % 2 else N // 2


def jackson_sigma(beta, n: int):
    b = np.abs(np.asarray(beta, dtype=np.float64))
    a = math.pi / (n + 1)
    s = ((n + 1 - b) * np.cos(a * b) + np.sin(a * b) / math.tan(a)) / (n + 1)
    return np.where(b <= n, s, 0.0)


def sigma_1d(N: int) -> np.ndarray:
    return jackson_sigma(modes_1d(N), jackson_n(N))


def sigma_nd(N: int, d: int) -> np.ndarray:
    s = sigma_1d(N)
    out = s
    for _ in range(d - 1):
        out = np.multiply.outer(out, s)
    return out.ravel()


def unfiltered_nd(N: int, d: int) -> np.ndarray:
    """The unfiltered method (sigma = 1) on the same mode set: for even N the
    modes with a component -N/2 are zeroed (section 4.1: even N reduces to
    the odd N - 1 case), as the filter itself does."""
    one = np.ones(N)
    if N % 2 == 0:
        one[modes_1d(N) == -(N // 2)] = 0.0
    out = one
    for _ in range(d - 1):
        out = np.multiply.outer(out, one)
    return out.ravel()


# ----------------------------------------------------------------------------
# Quadrature rules (library primitives: numpy's Gauss-Legendre nodes)
# ----------------------------------------------------------------------------

def gauss_legendre(n: int, a: float, b: float):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def directions_2d(M: int):
    """2M samples theta_t = t pi/(2M), t = 0..2M-1 on [0, pi): M samples in
    [0, pi/2) (section 4.2, Table 2 convention) plus their partners shifted by
    pi/2.  Returns (e_t, e_t^perp, weights pi/(2M)) -- eq. discrete_hatB."""
    th = np.arange(2 * M) * math.pi / (2 * M)
    e = np.stack([np.cos(th), np.sin(th)], axis=1)
    ep = np.stack([np.cos(th + math.pi / 2), np.sin(th + math.pi / 2)], axis=1)
    w = np.full(2 * M, math.pi / (2 * M))
    return e, ep, w


def hemisphere_split(M: int):
    """M = M_mu * M_phi with M_mu the largest divisor of M not above sqrt(M/2)."""
    best = 1
    for a in range(1, M + 1):
        if M % a == 0 and a * a <= M / 2.0:
            best = a
    return best, M // best


def directions_3d(M: int):
    """Hemisphere rule with positive weights summing to 2 pi: Gauss-Legendre
    in mu = cos(theta) on [-1,1] with 2 M_mu nodes, the positive half kept
    (integrands are even in e), times the uniform rule in azimuth."""
    mm, mp = hemisphere_split(M)
    x, w = np.polynomial.legendre.leggauss(2 * mm)
    keep = x > 0
    mu, wm = x[keep], w[keep]
    dirs, wts = [], []
    for i in range(mm):
        st = math.sqrt(max(0.0, 1.0 - mu[i] ** 2))
        for j in range(mp):
            ph = 2.0 * math.pi * j / mp
            dirs.append((st * math.cos(ph), st * math.sin(ph), mu[i]))
            wts.append(wm[i] * 2.0 * math.pi / mp)
    return np.array(dirs), np.array(wts)


# ----------------------------------------------------------------------------
# Kernel-mode factors by quadrature of their defining integrals
# ----------------------------------------------------------------------------

def _gl_nodes_for(omega_max: float, R: float):
    n = int(math.ceil(0.75 * omega_max * R)) + 48
    return gauss_legendre(n, -R, R)


def psi_line(s: np.ndarray, R: float, power: int) -> np.ndarray:
    """int_{-R}^{R} |rho|^power cos(rho s) d rho for each s (the imaginary part
    of int E_l(rho e) d rho vanishes by symmetry).  power=0 is psi_R of
    section 4.1 (2D); power=1 is its 3D analogue (Jacobian rho^{d-1} over
    the delta-function factor rho)."""
    smax = float(np.max(np.abs(s))) if s.size else 0.0
    # the integrand is even in rho (and has a kink at 0 when power = 1), so
    # integrate over [0, R] and double
    rho, w = _gl_nodes_for(smax, R)
    rho, w = 0.5 * (rho + R), 0.5 * w
    wt = 2.0 * w * rho ** power
    out = np.empty(s.shape)
    flat_s, flat_o = s.ravel(), out.ravel()
    for c0 in range(0, flat_s.size, 4096):
        blk = flat_s[c0:c0 + 4096]
        flat_o[c0:c0 + 4096] = np.cos(np.outer(blk, rho)) @ wt
    return out


def disk_integral(q: np.ndarray, R: float) -> np.ndarray:
    """Phi = 2 int_{|x|<=R, x in a plane} cos(q x_1) dx, the circle integral of
    psi_3 over the great circle orthogonal to e (the double cover of the disk
    gives the factor 2).  With x_1 = R cos(theta):
    Phi = 4 R^2 int_0^pi cos(q R cos theta) sin^2 theta d theta, evaluated by
    the periodic trapezoid rule (the integrand is smooth, even, 2pi-periodic)."""
    qmax = float(np.max(np.abs(q))) if q.size else 0.0
    K = 2 * int(math.ceil(qmax * R)) + 96
    th = 2.0 * math.pi * np.arange(K) / K
    ct, s2 = np.cos(th), np.sin(th) ** 2
    out = np.empty(q.shape)
    flat_q, flat_o = q.ravel(), out.ravel()
    for c0 in range(0, flat_q.size, 2048):
        blk = flat_q[c0:c0 + 2048]
        g = np.cos(np.outer(blk * R, ct)) @ s2
        flat_o[c0:c0 + 2048] = 4.0 * R * R * 0.5 * (2.0 * math.pi / K) * g
    return out


@dataclass
class LowRank:
    """B_fast(l, m) = sum_t c[t] U[t, l] V[t, m] over the modes of one grid."""
    c: np.ndarray       # (T,)
    U: np.ndarray       # (T, n)
    V: np.ndarray       # (T, n)

    def matrix(self) -> np.ndarray:
        return np.einsum("t,tl,tm->lm", self.c, self.U, self.V)

    def diagonal(self) -> np.ndarray:
        return np.einsum("t,tm,tm->m", self.c, self.U, self.V)


def lowrank_2d_maxwell(N: int, L: float, R: float, M: int) -> LowRank:
    """Section 4.1, eq. discrete_hatB with 2M samples on [0, pi), times the
    Maxwell constant Btilde = 2^{d-1} C_2 = 1/pi (section 1, eq. Carleman)."""
    kx, ky = mode_grid(N, 2)
    e, ep, w = directions_2d(M)
    bt = 2.0 * C_D[2]
    T = len(w)
    U = np.empty((T, kx.size)); V = np.empty((T, kx.size))
    for t in range(T):
        U[t] = psi_line(math.pi / L * (kx * e[t, 0] + ky * e[t, 1]), R, 0)
        V[t] = psi_line(math.pi / L * (kx * ep[t, 0] + ky * ep[t, 1]), R, 0)
    return LowRank(bt * w, U, V)


def lowrank_3d_hard_sphere(N: int, L: float, R: float, M: int) -> LowRank:
    """3D analogue of section 4.1: with y = rho e, z = rho* e* (rho in [-R,R],
    a double cover), B_hat = (Bt/4) int int delta(e.e*) psi_3(l,e) psi_3(m,e*)
    de de*; integrating e* over the great circle orthogonal to e gives
    B_hat = (Bt/2) int_{hemisphere} psi_3(l,e) Phi(m,e) de, discretised by the
    hemisphere rule.  Bt = 2^{d-1} C_3 |g|^{gamma+2-d} = 1/pi for gamma = 1."""
    kx, ky, kz = mode_grid(N, 3)
    dirs, w = directions_3d(M)
    bt = 4.0 * C_D[3]
    T = len(w)
    U = np.empty((T, kx.size)); V = np.empty((T, kx.size))
    kap2 = (kx * kx + ky * ky + kz * kz) * (math.pi / L) ** 2
    for t in range(T):
        s = math.pi / L * (kx * dirs[t, 0] + ky * dirs[t, 1] + kz * dirs[t, 2])
        U[t] = psi_line(s, R, 1)
        qperp = np.sqrt(np.maximum(kap2 - s * s, 0.0))
        V[t] = disk_integral(qperp, R)
    return LowRank(0.5 * bt * w, U, V)


def bcos_eval(bcos, x):
    """b(x) = sum_i bcos[i] x^i (b = 1 when bcos is empty or None)."""
    if not bcos:
        return np.ones_like(x)
    return np.polynomial.polynomial.polyval(x, np.asarray(bcos, float))


def hankel_disk(q: np.ndarray, rho: float, a: float, R: float, bcos=None) -> np.ndarray:
    """2 int_{|x|<=R, x in a plane} (rho^2 + |x|^2)^a b(cos theta) cos(q x_1) dx
    = 4 pi int_0^R (rho^2 + r^2)^a b(cos theta) J_0(q r) r dr (the angular
    integral of the disk is 2 pi J_0), by Gauss-Legendre in r.  rho > 0 keeps
    the weight smooth.  a = 0, b = 1 gives the hard-sphere disk integral.
    cos theta = (rho^2 - r^2)/(rho^2 + r^2) is the angle between g = y + z and
    w = (y - z)/|g| of the classical form for |y| = rho, |z| = r (y, z
    orthogonal)."""
    from scipy.special import j0
    qmax = float(np.max(np.abs(q))) if q.size else 0.0
    n = int(math.ceil(0.75 * qmax * R)) + 64
    # the weight varies on the scale rho near r = 0: split there
    rs = min(R, 8.0 * rho)
    r1, w1 = gauss_legendre(n, 0.0, rs)
    parts = [(r1, w1)]
    if rs < R:
        parts.append(gauss_legendre(n, rs, R))
    r = np.concatenate([x for x, _ in parts])
    w = np.concatenate([y for _, y in parts])
    wt = 4.0 * math.pi * w * r * (rho * rho + r * r) ** a
    wt = wt * bcos_eval(bcos, (rho * rho - r * r) / (rho * rho + r * r))
    out = np.empty(q.shape)
    flat_q, flat_o = q.ravel(), out.ravel()
    for c0 in range(0, flat_q.size, 2048):
        blk = flat_q[c0:c0 + 2048]
        flat_o[c0:c0 + 2048] = j0(np.outer(blk, r)) @ wt
    return out


def lowrank_3d_vhs(N: int, L: float, R: float, M: int, gamma: float, n_radial: int,
                   truncation: str = "box", bcos=None, modes=None) -> LowRank:
    """Variable hard spheres B = C_3 |g|^gamma in 3D: Carleman weight
    Bt(y, z) = 2^2 C_3 (|y|^2 + |z|^2)^a with a = (gamma - 1)/2 (section 1),
    which does not factor in (|y|, |z|).  The polar form of the 3D kernel
    (as for hard spheres) keeps the factor inside both radial integrals;
    discretising the radius of y by Gauss-Legendre (rho_j, omega_j) separates
    them (the form alpha_{l+m} beta_l gamma_m of section 4.1, here with
    M' = M n_radial terms):
        psi_{t,j}(l) = 2 omega_j rho_j cos(pi rho_j l.e_t / T),
        phi_{t,j}(m) = 2 int_{disk perp e_t, |x| <= r_j} (rho_j^2 + |x|^2)^a cos(pi m.x / T) dx,
    with the hemisphere rule over e_t and the constant (Bt/2) w_t as for hard
    spheres.  gamma = 1 reduces to the hard-sphere kernel as n_radial grows.

    truncation "box": |y| <= R and |z| <= R (the Carleman truncation of
    section 1.2): rho_j Gauss-Legendre on [0, R], r_j = R.
    truncation "ball": |y|^2 + |z|^2 = |g|^2 <= R^2, the truncation of the
    classical form (eq. classical_hatB: y = (g + |g| w)/2, z = (g - |g| w)/2
    are orthogonal with |y|^2 + |z|^2 = |g|^2): r_j = sqrt(R^2 - rho_j^2),
    with rho = R sin(theta) and Gauss-Legendre in theta on [0, pi/2] (the
    substitution removes the square-root endpoint of r_j).

    bcos: an angular factor B = C_3 |g|^gamma b(cos theta), b a polynomial
    (coefficients of 1, x, x^2, ...), inside the radial weight of phi_{t,j}
    (cos theta = (rho^2 - r^2)/(rho^2 + r^2), see hankel_disk).

    modes: optional (3, P) integer mode vectors at which to evaluate U and V
    (default: every mode of the grid, in the order of mode_grid).  The
    quadratures are sized by the largest frequency among the given modes."""
    kx, ky, kz = mode_grid(N, 3) if modes is None else (np.asarray(m, float) for m in modes)
    dirs, w = directions_3d(M)
    bt = 4.0 * C_D[3]
    a = 0.5 * (gamma - 1.0)
    if truncation == "box":
        rho, om = gauss_legendre(n_radial, 0.0, R)
        rdisk = np.full(n_radial, R)
    elif truncation == "ball":
        th, wt = gauss_legendre(n_radial, 0.0, 0.5 * math.pi)
        rho, om = R * np.sin(th), R * np.cos(th) * wt
        rdisk = R * np.cos(th)
    else:
        raise ValueError(f"truncation {truncation}")
    T = len(w)
    U = np.empty((T * n_radial, kx.size)); V = np.empty((T * n_radial, kx.size))
    c = np.empty(T * n_radial)
    kap2 = (kx * kx + ky * ky + kz * kz) * (math.pi / L) ** 2
    for t in range(T):
        s = math.pi / L * (kx * dirs[t, 0] + ky * dirs[t, 1] + kz * dirs[t, 2])
        qperp = np.sqrt(np.maximum(kap2 - s * s, 0.0))
        for j in range(n_radial):
            i = t * n_radial + j
            U[i] = 2.0 * om[j] * rho[j] * np.cos(rho[j] * s)
            V[i] = hankel_disk(qperp, rho[j], a, rdisk[j], bcos)
            c[i] = 0.5 * bt * w[t]
    return LowRank(c, U, V)


def ball_radial_integral(p: np.ndarray, q: np.ndarray, R: float) -> np.ndarray:
    """int_0^R rho^2 sinc(p rho) sinc(q rho) d rho (sinc x = sin x / x) for
    p, q >= 0, from the antiderivative of sin(p rho) sin(q rho) / (p q):
    R [sinc((p - q) R) - sinc((p + q) R)] / (2 p q); the limits p = 0 or
    q = 0 are int_0^R rho sin(x rho) / x d rho = (sin xR - xR cos xR) / x^3."""
    p, q = np.broadcast_arrays(np.asarray(p, float), np.asarray(q, float))
    out = np.empty(p.shape)
    sinc = lambda x: np.sinc(x / math.pi)
    both = (p > 0) & (q > 0)
    pp, qq = p[both], q[both]
    out[both] = R * (sinc((pp - qq) * R) - sinc((pp + qq) * R)) / (2.0 * pp * qq)
    for one, x in (((p > 0) & (q == 0), p), ((p == 0) & (q > 0), q)):
        xx = x[one]
        out[one] = (np.sin(xx * R) - xx * R * np.cos(xx * R)) / xx ** 3
    out[(p == 0) & (q == 0)] = R ** 3 / 3.0
    return out


def classical_kernel_3d_angular(N: int, L: float, R: float, bcos, gamma: float = 0.0,
                                n_rho: int = 96) -> np.ndarray:
    """Dense classical-form modes (eq. classical_hatB) for B = C_3 |g|^gamma
    b(g.w / |g|), b a polynomial, by the Funk-Hecke formula: with
    b = sum_n beta_n P_n (Legendre coefficients), the sphere integral of
    b(g^.w) E over w is 4 pi sum_n beta_n i^n j_n(a |g| |l-m|) P_n(g^.u), and
    the sphere integral over g^ then gives
        B(l,m) = C_3 (4 pi)^2 sum_n beta_n (-1)^n P_n(cos phi)
                 int_0^R rho^{2+gamma} j_n(a rho |l+m|) j_n(a rho |l-m|) d rho,
    cos phi = (|l|^2 - |m|^2) / (|l+m| |l-m|), a = pi / (2T); the radial
    integral by Gauss-Legendre (n_rho nodes).  b = 1 is classical_kernel_3d."""
    from scipy.special import eval_legendre, spherical_jn
    beta = np.polynomial.legendre.poly2leg(np.asarray(bcos, float))
    k = np.array(mode_grid(N, 3), dtype=float).T
    n = k.shape[0]
    a = math.pi / (2.0 * L)
    rho, w = gauss_legendre(n_rho, 0.0, R)
    wr = w * rho ** (2.0 + gamma)
    B = np.zeros((n, n))
    for i0 in range(0, n, 64):
        l = k[i0:i0 + 64, None, :]
        sp = np.sqrt(((l + k[None]) ** 2).sum(axis=2))
        sm = np.sqrt(((l - k[None]) ** 2).sum(axis=2))
        num = (l * l).sum(axis=2) - (k[None] * k[None]).sum(axis=2)
        den = sp * sm
        cphi = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
        blk = np.zeros(sp.shape)
        for nn, bn in enumerate(beta):
            if bn == 0.0:
                continue
            jp = spherical_jn(nn, a * sp[..., None] * rho)
            jm = spherical_jn(nn, a * sm[..., None] * rho)
            blk += bn * (-1.0) ** nn * eval_legendre(nn, cphi) * ((jp * jm) @ wr)
        B[i0:i0 + 64] = C_D[3] * (4.0 * math.pi) ** 2 * blk
    return B


def classical_kernel_3d(N: int, L: float, R: float) -> np.ndarray:
    """Dense kernel modes of the classical form (eq. classical_hatB) for 3D
    Maxwell molecules, B = C_3: the sphere integral of E over w is
    4 pi sinc(a |g| |l - m|) and then the ball integral of E_{l+m}(g/2)
    gives
        B(l, m) = C_3 (4 pi)^2 int_0^R rho^2 sinc(a rho |l+m|) sinc(a rho |l-m|) d rho,
    a = pi / (2 T).  Exact (no direction or radial quadrature); n x n in the
    mode order of mode_grid, for small grids."""
    k = np.array(mode_grid(N, 3), dtype=float).T
    n = k.shape[0]
    a = math.pi / (2.0 * L)
    B = np.empty((n, n))
    for i0 in range(0, n, 256):
        l = k[i0:i0 + 256, None, :]
        sp = np.sqrt(((l + k[None]) ** 2).sum(axis=2))
        sm = np.sqrt(((l - k[None]) ** 2).sum(axis=2))
        B[i0:i0 + 256] = C_D[3] * (4.0 * math.pi) ** 2 * ball_radial_integral(a * sp, a * sm, R)
    return B


# ----------------------------------------------------------------------------
# Plan
# ----------------------------------------------------------------------------

@dataclass
class Plan:
    N: int
    d: int
    L: float
    R: float
    M: int
    kind: str
    sigma: np.ndarray
    lr: LowRank
    # None: sigma and the low-rank factors cover every mode (mode_grid order).
    # Otherwise (d, S) integer mode vectors: they cover only these modes, and
    # the plan serves inputs whose spectrum vanishes off them (collide_points).
    modes: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.N ** self.d

    @property
    def h(self) -> float:
        return 2.0 * self.L / self.N


def make_plan(N: int, d: int, L: float, M: int, kind: str | None = None,
              R: float = 6.0, filtered: bool = True, gamma: float | None = None,
              n_radial: int = 8, truncation: str = "box", bcos=None, modes=None) -> Plan:
    """kind None: 2D Maxwell / 3D hard spheres.  In 3D, KIND_MAXWELL is the
    variable-hard-sphere kernel with gamma = 0 and KIND_VHS takes gamma; both
    use n_radial radial nodes (M' = M n_radial terms) and either truncation
    (lowrank_3d_vhs).  modes: optional (d, S) integer mode vectors in [-N/2,
    N/2) (3D radial kernels only): the plan then holds the filter and the
    low-rank factors on these modes only, for inputs whose spectrum lives on
    them (collide_points), so that large grids with many products stay cheap."""
    if modes is not None:
        if not (d == 3 and kind in (KIND_MAXWELL, KIND_VHS)):
            raise NotImplementedError("a mode subset needs the 3D radial (non-separable) path")
        modes = np.asarray(modes, dtype=np.int64)
        g = 0.0 if kind == KIND_MAXWELL else float(gamma)
        lr = lowrank_3d_vhs(N, L, R, M, g, n_radial, truncation, bcos, modes=modes)
        s1 = sigma_1d(N) if filtered else unfiltered_nd(N, 1)
        sig = np.prod([s1[m % N] for m in modes], axis=0)
        return Plan(N, d, L, R, M, kind, sig, lr, modes)
    if kind is None:
        kind = KIND_MAXWELL if d == 2 else KIND_HARD_SPHERE
    if d == 2 and kind == KIND_MAXWELL:
        lr = lowrank_2d_maxwell(N, L, R, M)
    elif d == 3 and kind == KIND_HARD_SPHERE:
        lr = lowrank_3d_hard_sphere(N, L, R, M)
    elif d == 3 and kind in (KIND_MAXWELL, KIND_VHS):
        g = 0.0 if kind == KIND_MAXWELL else float(gamma)
        lr = lowrank_3d_vhs(N, L, R, M, g, n_radial, truncation, bcos)
    else:
        raise NotImplementedError(f"oracle kernel {kind} in {d}D")
    if (truncation != "box" or bcos) and not (d == 3 and kind in (KIND_MAXWELL, KIND_VHS)):
        raise NotImplementedError("the ball truncation and an angular factor need the radial "
                                  "(non-separable) path")
    sig = sigma_nd(N, d) if filtered else unfiltered_nd(N, d)
    return Plan(N, d, L, R, M, kind, sig, lr)


# ----------------------------------------------------------------------------
# Collision term: direct double sum (section 3.2.2, eq. Qsk and eq. Qsr)
# ----------------------------------------------------------------------------

def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        _lib.efm_direct_sum.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + [dp] * 10
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Collision:
    Q: np.ndarray
    Qplus: np.ndarray
    Qminus: np.ndarray
    imag_max: float
    Qhat: np.ndarray


def collide_modes(plan: Plan, F: np.ndarray) -> Collision:
    """Q^sigma on the grid from the plain double sum over modes."""
    lib = _load()
    Fh = dft(F, plan.L).ravel()
    Fr = np.ascontiguousarray(Fh.real); Fi = np.ascontiguousarray(Fh.imag)
    U = np.ascontiguousarray(plan.lr.U.T); V = np.ascontiguousarray(plan.lr.V.T)
    c = np.ascontiguousarray(plan.lr.c); sig = np.ascontiguousarray(plan.sigma)
    n = plan.n
    Gr, Gi, Lr, Li = (np.empty(n) for _ in range(4))
    lib.efm_direct_sum(plan.d, plan.N, len(c), _p(c), _p(U), _p(V), _p(sig),
                       _p(Fr), _p(Fi), _p(Gr), _p(Gi), _p(Lr), _p(Li))
    shp = (plan.N,) * plan.d
    G = (Gr + 1j * Gi).reshape(shp)
    Lh = (Lr + 1j * Li).reshape(shp)
    qp = idft(G, plan.L); qm = idft(Lh, plan.L)
    q = qp - qm
    imag = float(max(np.abs(qp.imag).max(), np.abs(qm.imag).max()))
    return Collision(q.real, qp.real, qm.real, imag, G - Lh)


def collide_dense(B: np.ndarray, sigma: np.ndarray, F: np.ndarray, L: float) -> np.ndarray:
    """Q^sigma on the grid (section 3.2.2, eq. EFMk) from a dense kernel-mode
    matrix B (mode order of mode_grid): Qh_k = sum_{l + m = k mod N}
    (sigma_l sigma_m B(l,m) - sigma_m^2 B(m,m)) Fh_l Fh_m, summed with numpy
    over l for every output mode k."""
    N, d = F.shape[0], F.ndim
    n = N ** d
    Bs = B * sigma[:, None] * sigma[None, :]
    diag = np.diag(Bs).copy()
    pos = np.array(mode_grid(N, d)).T % N
    Fh = dft(F, L).ravel()
    Qh = np.empty(n, complex)
    ar = np.arange(n)
    for k in range(n):
        mp = (pos[k] - pos) % N
        m = mp[:, 0]
        for i in range(1, d):
            m = m * N + mp[:, i]
        pr = Fh * Fh[m]
        Qh[k] = np.dot(Bs[ar, m] - diag[m], pr)
    return idft(Qh.reshape((N,) * d), L).real


def collision_frequency(plan: Plan, F: np.ndarray) -> np.ndarray:
    """l_r with Q-_r = F_r l_r: l_r = sum_m B^s(m,m) Fh_m E_m(r) (the loss
    identity of section 3.1.2, with the filtered kernel)."""
    Fh = dft(F, plan.L).ravel()
    D = plan.sigma * plan.sigma * plan.lr.diagonal()
    return idft((D * Fh).reshape(F.shape), plan.L).real


# ----------------------------------------------------------------------------
# Point-by-point evaluation through the factorised fast algorithm
# (section 3.1.1, eq. fastFGM with the collocation evaluation eq. FGM_Qcv;
#  filtered as in section 4.1).  Explicit exponential sums, no FFT.
# ----------------------------------------------------------------------------

def collide_points(plan: Plan, F: np.ndarray, idx: np.ndarray):
    """Q, Q+ and Q- at the flat grid indices idx.

    a_t(r) = sum_k sig_k U_t(k) Fh_k E_k(r),  b_t(r) = sum_k sig_k V_t(k) Fh_k E_k(r)
    Q+(r)  = sum_t c_t a_t(r) b_t(r)
    l(r)   = sum_k sig_k^2 (sum_t c_t U_t(k) V_t(k)) Fh_k E_k(r),  Q-(r) = F_r l(r)
    """
    Fh = dft(F, plan.L).ravel()
    kl = mode_grid(plan.N, plan.d)
    if plan.modes is not None:
        # the spectrum must vanish off the plan's modes (to roundoff): then
        # the sums over all modes are the sums over these
        N = plan.N
        flat = np.zeros(plan.modes.shape[1], dtype=np.int64)
        for m in plan.modes:
            flat = flat * N + (m % N)
        if np.unique(flat).size != flat.size:
            raise ValueError("repeated modes in the plan")
        off = np.ones(plan.n, bool)
        off[flat] = False
        if np.abs(Fh[off]).max(initial=0.0) > 1e-13 * np.abs(Fh).max():
            raise ValueError("the input's spectrum does not vanish off the plan's modes")
        Fh = Fh[flat]
        kl = list(plan.modes)
    vl = [v[idx] for v in grid_points(plan.N, plan.d, plan.L)]
    Er = E(kl, vl, plan.L)                       # (P, n)
    sF = plan.sigma * Fh
    A = Er @ (plan.lr.U * sF).T                  # (P, T)
    B = Er @ (plan.lr.V * sF).T
    qp = (A * B) @ plan.lr.c
    ell = Er @ (plan.sigma * plan.sigma * plan.lr.diagonal() * Fh)
    qm = F.ravel()[idx] * ell
    return (qp - qm).real, qp.real, qm.real, float(np.abs(qp.imag).max() + np.abs(ell.imag).max())


# ----------------------------------------------------------------------------
# DVM form on tiny grids (section 3.2, eq. A_simplified, eq. tildetildeA,
# eq. Qsr)
# ----------------------------------------------------------------------------

def kernel_matrix(plan: Plan, symmetrise: bool = True) -> np.ndarray:
    B = plan.lr.matrix()
    if symmetrise:
        B = 0.5 * (B + B.T)
    return plan.sigma[:, None] * B * plan.sigma[None, :]


def G_sigma(plan: Plan, symmetrise: bool = True) -> np.ndarray:
    """G(a, b) = sum_{i,j in K} B^s(i,j) E_{-i}(h a) E_{-j}(h b) on grid index
    differences a, b (section 3.2.1, eq. G and section 3.2.2, eq. tildeG without
    the 1/N^{2d} factor, which the caller applies)."""
    kl = mode_grid(plan.N, plan.d)
    h = plan.h
    idx = np.arange(plan.N)            # index differences a in [0, N), offset a*h
    al = [x.ravel() * h for x in np.meshgrid(*([idx] * plan.d), indexing="ij")]
    Em = np.conj(E(kl, al, plan.L))                   # E_{-i}(a h): (points, modes)
    return Em @ kernel_matrix(plan, symmetrise) @ Em.T


def dvm_tensor(plan: Plan, symmetrise: bool = True) -> np.ndarray:
    """A[r, s, p, q] = N^{-2d} 1_N(r+s-p-q) G(p-s, q-s)."""
    n, N, d = plan.n, plan.N, plan.d
    G = G_sigma(plan, symmetrise)
    coords = np.stack(np.unravel_index(np.arange(n), (N,) * d), axis=1)

    def flat(c):
        return np.ravel_multi_index(tuple((c % N).T), (N,) * d)

    A = np.zeros((n, n, n, n))
    G = G.real
    allp = np.arange(n)
    for r in range(n):
        for s in range(n):
            q = flat(coords[r] + coords[s] - coords)            # all p at once
            A[r, s, allp, q] = G[flat(coords - coords[s]), flat(coords[q] - coords[s])]
    return A / n ** 2


def collide_dvm(A: np.ndarray, F: np.ndarray) -> np.ndarray:
    f = F.ravel()
    gain = np.einsum("rspq,p,q->r", A, f, f)
    loss = np.einsum("rspq,r,s->r", A, f, f)
    return (gain - loss).reshape(F.shape)


# ----------------------------------------------------------------------------
# Diagnostics (Theorem 1; section 4.2: positivity error epsilon, entropy eta)
# ----------------------------------------------------------------------------

def monitors(plan: Plan, F: np.ndarray, Q: np.ndarray) -> dict:
    h = plan.h ** plan.d
    f = F.ravel(); q = Q.ravel()
    pos = f > 0
    V = grid_points(plan.N, plan.d, plan.L)
    return {
        "mass": h * f.sum(),
        "sumQ": q.sum(),
        "sumabsQ": np.abs(q).sum(),
        "entropy_prod": h * np.sum(q[pos] * np.log(f[pos])),
        "eta": h * np.sum(f[pos] * np.log(f[pos])),
        "minF": f.min(),
        "n_nonpos": int((~pos).sum()),
        "eps_pos": (np.abs(f).sum() - f.sum()) / np.abs(f).sum(),
        "momentum": [h * np.sum(q * v) for v in V],
        "energy": h * np.sum(q * sum(v * v for v in V)),
    }


def fe_step(L_op, F, dt):
    return F + dt * L_op(F)


def ssprk3_step(L_op, F, dt):
    """Third-order SSP Runge-Kutta (section 4.1), Shu-Osher form."""
    u1 = F + dt * L_op(F)
    u2 = 0.75 * F + 0.25 * (u1 + dt * L_op(u1))
    return F / 3.0 + 2.0 / 3.0 * (u2 + dt * L_op(u2))


# ----------------------------------------------------------------------------
# Closed forms used as pins
# ----------------------------------------------------------------------------

def bkw_S(d: int, t: float) -> float:
    return 1.0 - math.exp(-t / 8.0) / 2.0 if d == 2 else 1.0 - 2.0 * math.exp(-t / 6.0) / 5.0


def bkw_f(d: int, t: float, v2: np.ndarray) -> np.ndarray:
    """BKW solution (section 4.2, Example 1 in 2D, Example 4 in 3D)."""
    S = bkw_S(d, t)
    if d == 2:
        return (1 / (2 * math.pi * S) * np.exp(-v2 / (2 * S))
                * ((2 * S - 1) / S + (1 - S) / (2 * S * S) * v2))
    return ((2 * math.pi * S) ** -1.5 * np.exp(-v2 / (2 * S))
            * ((5 * S - 3) / (2 * S) + (1 - S) / (2 * S * S) * v2))


def bkw_dfdt(d: int, t: float, v2: np.ndarray) -> np.ndarray:
    """d f / d t of the BKW solution = (df/dS)(dS/dt), differentiated by hand."""
    S = bkw_S(d, t)
    if d == 2:
        dS = math.exp(-t / 8.0) / 16.0
        g = np.exp(-v2 / (2 * S))
        P = (2 * S - 1) / S + (1 - S) / (2 * S * S) * v2
        dP = 1.0 / (S * S) + v2 * (-1.0 / (2 * S * S) - (1 - S) / S ** 3)
        pref = 1 / (2 * math.pi * S)
        dpref = -1 / (2 * math.pi * S * S)
        dg = g * v2 / (2 * S * S)
        return (dpref * g * P + pref * dg * P + pref * g * dP) * dS
    dS = 2.0 * math.exp(-t / 6.0) / 30.0
    g = np.exp(-v2 / (2 * S))
    P = (5 * S - 3) / (2 * S) + (1 - S) / (2 * S * S) * v2
    dP = 3.0 / (2 * S * S) + v2 * (-1.0 / (2 * S * S) - (1 - S) / S ** 3)
    pref = (2 * math.pi * S) ** -1.5
    dpref = -1.5 * (2 * math.pi) ** -1.5 * S ** -2.5
    dg = g * v2 / (2 * S * S)
    return (dpref * g * P + pref * dg * P + pref * g * dP) * dS

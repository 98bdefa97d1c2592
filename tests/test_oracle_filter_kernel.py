"""Pins of the oracle's filter and kernel-mode tables against facts fixed by
the paper and by mathematics (not by retyping the oracle's formulas)."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as sp

from oracle import efm

R = 6.0
T_PAPER = efm.default_box(R)


# --------------------------------------------------------------------------
# Modified Jackson filter (section 3.2.2, eq. JacksonFilter2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [3, 7, 8, 15, 16, 31, 32])
def test_jackson_is_sine_window_autocorrelation(n):
    """sigma_n(beta) equals the normalised autocorrelation of the window
    a_j = sin(pi j/(n+1)), j = 1..n; so its trigonometric polynomial is
    |sum_j a_j e^{i j x}|^2 / |a|^2 >= 0 (why the filter restores positivity)."""
    a = np.sin(np.pi * np.arange(1, n + 1) / (n + 1))
    ac = np.array([np.dot(a[: n - b], a[b:]) for b in range(n + 1)]) / np.dot(a, a)
    s = efm.jackson_sigma(np.arange(n + 1), n)
    assert np.abs(ac - s).max() < 1e-14


@pytest.mark.parametrize("N", [15, 16, 32, 33, 64])
def test_jackson_special_values(N):
    s = efm.sigma_1d(N)
    k = efm.modes_1d(N)
    n = efm.jackson_n(N)
    assert s[k == 0][0] == pytest.approx(1.0, abs=1e-15)
    assert s[k == 1][0] == pytest.approx(math.cos(math.pi / (n + 1)), abs=1e-15)
    assert np.all(s >= -1e-15) and np.all(s <= 1.0 + 1e-15)
    assert np.allclose(s[np.abs(k) >= n], 0.0, atol=1e-15)
    if N % 2 == 0:
        assert s[k == -N // 2][0] == pytest.approx(0.0, abs=1e-15)
    # even: sigma(-k) = sigma(k) wherever both modes exist
    for kk in range(1, (N - 1) // 2 + 1):
        assert s[k == kk][0] == pytest.approx(s[k == -kk][0], abs=0)


@pytest.mark.parametrize("N", [16, 17, 32])
def test_filtered_dirichlet_kernel_nonnegative(N):
    """chi^sigma_N(v) = sum_k sigma(k) E_k(v) >= 0 on a 64x refined grid, while
    the unfiltered Dirichlet kernel chi_N takes negative values (3.2.1-3.2.2)."""
    k = efm.modes_1d(N)
    x = np.linspace(-math.pi, math.pi, 64 * N, endpoint=False)
    chi_s = np.real(np.exp(1j * np.outer(x, k)) @ efm.sigma_1d(N))
    chi = np.real(np.exp(1j * np.outer(x, k)) @ np.ones(N))
    assert chi_s.min() > -1e-12 * chi_s.max()
    assert chi.min() < -0.05 * chi.max()


# --------------------------------------------------------------------------
# Kernel-mode factors vs closed forms from independent library routines
# --------------------------------------------------------------------------

def test_psi_line_closed_forms():
    s = np.concatenate([[0.0], np.linspace(1e-3, 12.0, 257), -np.linspace(0.5, 9.0, 17)])
    p0 = efm.psi_line(s, R, 0)
    p1 = efm.psi_line(s, R, 1)
    with np.errstate(invalid="ignore", divide="ignore"):
        ref0 = np.where(s == 0, 2 * R, 2 * np.sin(R * s) / s)
        ref1 = np.where(s == 0, R * R, 2 * (R * np.sin(R * s) / s + (np.cos(R * s) - 1) / s ** 2))
    assert np.abs(p0 - ref0).max() < 1e-12 * 2 * R
    assert np.abs(p1 - ref1).max() < 1e-12 * R * R
    assert p0[0] == pytest.approx(2 * R, rel=1e-15)
    assert p1[0] == pytest.approx(R * R, rel=1e-15)


def test_disk_integral_bessel():
    q = np.concatenate([[0.0], np.linspace(1e-3, 14.0, 301)])
    ph = efm.disk_integral(q, R)
    with np.errstate(invalid="ignore", divide="ignore"):
        ref = np.where(q == 0, 2 * math.pi * R * R, 4 * math.pi * R * sp.j1(q * R) / q)
    assert np.abs(ph - ref).max() < 1e-12 * 2 * math.pi * R * R


@pytest.mark.parametrize("M", [1, 2, 3, 16])
def test_kernel_zero_mode_2d(M):
    """B_hat(0,0) = int int Bt delta(y.z) over B_R x B_R = (1/pi)(2R)^2 pi = 4 R^2."""
    p = efm.make_plan(8, 2, T_PAPER, M, R=R)
    B = p.lr.matrix()
    assert B[0, 0] == pytest.approx(4 * R * R, rel=1e-14)


@pytest.mark.parametrize("M", [2, 8, 32])
def test_kernel_zero_mode_3d(M):
    """3D hard spheres: int_{B_R} dy int_{B_R} delta(y.z) dz = int pi R^2/|y| dy
    = 2 pi^2 R^4, times Bt = 1/pi."""
    p = efm.make_plan(4, 3, 8.0, M, R=R)
    assert p.lr.diagonal()[0] == pytest.approx(2 * math.pi * R ** 4, rel=1e-14)


def test_hemisphere_rule():
    for M in [8, 16, 32, 64]:
        e, w = efm.directions_3d(M)
        assert len(w) == M and np.all(w > 0)
        assert w.sum() == pytest.approx(2 * math.pi, rel=1e-14)
        assert np.allclose(np.linalg.norm(e, axis=1), 1.0, atol=1e-15)
        assert np.all(e[:, 2] > 0)
        # even polynomials integrate exactly: int_{S2+} z^2 = int x^2 = 2 pi/3
        assert (w * e[:, 2] ** 2).sum() == pytest.approx(2 * math.pi / 3, rel=1e-13)
        assert (w * e[:, 0] ** 2).sum() == pytest.approx(2 * math.pi / 3, rel=1e-13)


def test_kernel_symmetries():
    p2 = efm.make_plan(8, 2, T_PAPER, 3, R=R)
    B = p2.lr.matrix()
    k = efm.mode_grid(8, 2)
    n = B.shape[0]
    neg = np.array([np.ravel_multi_index(((-k[0][i]) % 8, (-k[1][i]) % 8), (8, 8)) for i in range(n)])
    ok = np.array([abs(k[0][i]) < 4 and abs(k[1][i]) < 4 for i in range(n)])
    assert np.abs(B - B.T).max() < 1e-12 * B.max()
    Bs = B[np.ix_(ok, ok)]
    assert np.abs(Bs - B[np.ix_(ok, neg[ok])]).max() < 1e-12 * B.max()
    p3 = efm.make_plan(4, 3, 8.0, 8, R=R)
    B3 = p3.lr.matrix()
    k3 = efm.mode_grid(4, 3)
    n3 = B3.shape[0]
    neg3 = np.array([np.ravel_multi_index(tuple((-k3[j][i]) % 4 for j in range(3)), (4, 4, 4)) for i in range(n3)])
    ok3 = np.array([all(abs(k3[j][i]) < 2 for j in range(3)) for i in range(n3)])
    assert np.abs(B3[np.ix_(ok3, ok3)] - B3[np.ix_(ok3, neg3[ok3])]).max() < 1e-10 * B3.max()
    assert np.abs(B3[np.ix_(ok3, ok3)] - B3[np.ix_(neg3[ok3], ok3)]).max() < 1e-10 * B3.max()


def _exact_2d(l, m, L):
    """B_hat(l,m) = (1/pi) int_0^pi psi(l,e_th) psi(m, e_{th+pi/2}) d th
    (section 4.1, eq. fast_hatB, with Bt = 1/pi), psi = 2 sin(R s)/s."""
    def psi(k, th):
        s = math.pi / L * (k[0] * math.cos(th) + k[1] * math.sin(th))
        return 2 * R if abs(s) < 1e-300 else 2 * math.sin(R * s) / s

    def f(th):
        return psi(l, th) * psi(m, th + math.pi / 2)
    val, _ = si.quad(f, 0.0, math.pi, limit=400, epsabs=1e-13, epsrel=1e-13)
    return val / math.pi


def test_kernel_2d_converges_to_exact_integral():
    pairs = [((1, 0), (0, 2)), ((3, -2), (1, 1)), ((2, 5), (-4, 3)), ((0, 0), (6, 1))]
    errs = []
    for M in [4, 8, 16, 32]:
        p = efm.make_plan(16, 2, T_PAPER, M, R=R)
        B = p.lr.matrix()
        e = 0.0
        for l, m in pairs:
            il = np.ravel_multi_index((l[0] % 16, l[1] % 16), (16, 16))
            im = np.ravel_multi_index((m[0] % 16, m[1] % 16), (16, 16))
            e = max(e, abs(B[il, im] - _exact_2d(l, m, T_PAPER)) / (4 * R * R))
        errs.append(e)
    assert errs[-1] < 1e-9
    assert errs[0] > errs[1] > errs[2]


def test_kernel_3d_zero_row_converges_to_closed_form():
    """B_hat(0,m) = Bt int_{B_R} E_m(z) pi R^2/|z| dz = 4 pi R^2 (1 - cos kR)/k^2
    with k = pi|m|/L; by the symmetry of the continuous kernel B_hat(l,0) is the
    same function of l.  The low-rank rule converges to it as M grows."""
    L = 8.0
    N = 8
    k = efm.mode_grid(N, 3)
    kap = math.pi / L * np.sqrt(k[0] ** 2 + k[1] ** 2 + k[2] ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        ref = np.where(kap == 0, 2 * math.pi * R ** 4, 4 * math.pi * R * R * (1 - np.cos(kap * R)) / kap ** 2)
    errs_row, errs_col = [], []
    for M in [8, 32, 128, 512]:
        p = efm.make_plan(N, 3, L, M, R=R)
        row = np.einsum("t,t,tm->m", p.lr.c, p.lr.U[:, 0], p.lr.V)
        col = np.einsum("t,tl,t->l", p.lr.c, p.lr.U, p.lr.V[:, 0])
        errs_row.append(np.abs(row - ref).max() / ref.max())
        errs_col.append(np.abs(col - ref).max() / ref.max())
    assert errs_row[-1] < 1e-6 and errs_col[-1] < 1e-6
    assert errs_row[0] > errs_row[-1] and errs_col[0] > errs_col[-1]


def test_kernel_2d_zero_row_closed_form():
    """2D: B_hat(0,m) = (1/pi) int_{B_R} (2R/|z|) E_m(z) dz = 4R int_0^R J0(k r) dr."""
    N = 16
    p = efm.make_plan(N, 2, T_PAPER, 32, R=R)
    k = efm.mode_grid(N, 2)
    row = np.einsum("t,t,tm->m", p.lr.c, p.lr.U[:, 0], p.lr.V)
    for i in [1, 5, 17, 40, 77, 130]:
        kap = math.pi / T_PAPER * math.hypot(k[0][i], k[1][i])
        ref = 4 * R * si.quad(lambda r: sp.j0(kap * r), 0, R, limit=200, epsabs=1e-14)[0]
        assert row[i] == pytest.approx(ref, rel=1e-7, abs=1e-9 * 4 * R * R)

"""Pins of the oracle's collision term: independent formulations agree, the
invariants of Theorem 1 hold, and the paper's printed numbers are reproduced."""
import math

import numpy as np
import pytest

import synth
from oracle import efm

R = 6.0
T_PAPER = efm.default_box(R)


def _mix(seed, d, N, L):
    return synth.sample_mixture(synth.mixture_two_gaussians(seed, d), N, L)


# --------------------------------------------------------------------------
# Two formulations of the same operator (section 3.1-3.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,N,M,L", [(2, 4, 3, T_PAPER), (2, 6, 2, T_PAPER), (3, 4, 8, 8.0)])
def test_dvm_equals_mode_sum(d, N, M, L):
    """Brute-force DVM form (eq. A_simplified with the filtered kernel, eq.
    Qsr) equals the Fourier form (eq. Qsk) on tiny grids."""
    p = efm.make_plan(N, d, L, M, R=R)
    F = _mix(11 + N, d, N, L) + 0.01
    A = efm.dvm_tensor(p)
    q_dvm = efm.collide_dvm(A, F)
    c = efm.collide_modes(p, F)
    scale = np.abs(c.Qplus).max()
    assert np.abs(q_dvm - c.Q).max() < 1e-12 * scale
    # coefficient properties of Condition 1 (section 2): A >= 0 and symmetric
    assert A.min() > -1e-13 * A.max()
    assert np.abs(A - A.transpose(0, 1, 3, 2)).max() < 1e-13 * A.max()
    assert np.abs(A - A.transpose(2, 3, 0, 1)).max() < 1e-13 * A.max()


def test_unfiltered_G_has_negative_values_filtered_not():
    """Section 3.2.1, Figure 1: G(y, z) for N = 32 at z = (T/2, T/2), Bt = 1/pi,
    R = 6 in 2D has negative values; with the Jackson filter (section 3.2.2)
    G^sigma >= 0."""
    N = 32
    pu = efm.make_plan(N, 2, T_PAPER, 32, R=R, filtered=False)
    pf = efm.make_plan(N, 2, T_PAPER, 32, R=R, filtered=True)
    b = np.ravel_multi_index((N // 4, N // 4), (N, N))     # z = (T/2, T/2)
    Gu = efm.G_sigma(pu)[:, b].real
    Gf = efm.G_sigma(pf)[:, b].real
    assert Gu.min() < -1e-2 * Gu.max()
    assert Gf.min() > -1e-10 * Gf.max()


@pytest.mark.parametrize("d,N,M,L", [(2, 16, 4, T_PAPER), (3, 8, 8, 8.0), (3, 10, 32, 8.0)])
def test_pointwise_fast_algorithm_equals_mode_sum(d, N, M, L):
    """The factorised fast algorithm (eq. fastFGM / eq. fastAlg, filtered)
    evaluated by explicit exponential sums equals the double sum."""
    p = efm.make_plan(N, d, L, M, R=R)
    F = _mix(21 + N, d, N, L)
    c = efm.collide_modes(p, F)
    idx = np.random.default_rng(5).choice(p.n, 23, replace=False)
    q, qp, qm, imag = efm.collide_points(p, F, idx)
    scale = np.abs(c.Qplus).max()
    assert np.abs(q - c.Q.ravel()[idx]).max() < 1e-13 * scale
    assert np.abs(qp - c.Qplus.ravel()[idx]).max() < 1e-13 * scale
    assert imag < 1e-13 * scale


# --------------------------------------------------------------------------
# Theorem 1 and the sign structure
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d,N,M,L", [(2, 32, 16, 8.0), (3, 12, 32, 8.0)])
def test_mass_and_h_theorem(d, N, M, L):
    p = efm.make_plan(N, d, L, M, R=R)
    for seed in range(3):
        F = synth.sample_mixture(synth.mixture_anisotropic(100 + seed, d), N, L)
        c = efm.collide_modes(p, F)
        m = efm.monitors(p, F, c.Q)
        # mass (eq. conservationMass): Qhat_0 = 0
        assert abs(m["sumQ"]) < 1e-13 * m["sumabsQ"]
        # discrete H-theorem (eq. Htheorem)
        assert m["entropy_prod"] <= 0.0
        # gain and collision frequency are non-negative (A^sigma >= 0)
        assert c.Qplus.min() > -1e-12 * c.Qplus.max()
        ell = efm.collision_frequency(p, F)
        assert ell.min() > -1e-12 * ell.max()
        assert np.abs(F * ell - c.Qminus).max() < 1e-13 * np.abs(c.Qminus).max()
        assert c.imag_max < 1e-14 * np.abs(c.Qplus).max()


@pytest.mark.parametrize("d,N,M,L", [(2, 16, 8, 8.0), (2, 10, 4, 8.0), (3, 8, 8, 8.0), (3, 6, 8, 8.0)])
def test_unfiltered_even_n_zeroing_pins_mass(d, N, M, L):
    """The unfiltered method (sigma = 1) on even N: section 4.1 reduces even N
    to the odd N - 1 case by zeroing the kernel on modes with a component
    -N/2.  With that zeroing the discrete mass is conserved exactly (Theorem
    1, eq. conservationMass: Qhat_0 = 0 needs B(-m, m) = B(m, m), and -m of a
    mode with a component -N/2 wraps to itself mod N).  Keeping those modes
    breaks it: a planted sigma = 1 everywhere must lose mass."""
    p = efm.make_plan(N, d, L, M, R=R, filtered=False)
    # the zeroed modes are exactly those with some component -N/2
    kl = np.array(efm.mode_grid(N, d))
    has_edge = np.any(kl == -(N // 2), axis=0)
    assert np.all(p.sigma[has_edge] == 0.0) and np.all(p.sigma[~has_edge] == 1.0)
    for seed in range(2):
        F = synth.sample_mixture(synth.mixture_anisotropic(300 + seed, d), N, L)
        c = efm.collide_modes(p, F)
        m = efm.monitors(p, F, c.Q)
        assert abs(m["sumQ"]) <= 1e-13 * m["sumabsQ"]
        # the planted mistake: no zeroing of the -N/2 modes
        bad = efm.Plan(p.N, p.d, p.L, p.R, p.M, p.kind, np.ones(p.n), p.lr)
        cb = efm.collide_modes(bad, F)
        mb = efm.monitors(bad, F, cb.Q)
        assert abs(mb["sumQ"]) > 1e-6 * mb["sumabsQ"]


def test_gain_nonnegative_where_f_vanishes():
    """Proof of Theorem 1: where F_r = 0, dF_r/dt = sum A F_p F_q >= 0."""
    N, L = 16, 8.0
    p = efm.make_plan(N, 2, L, 8, R=R)
    F = _mix(7, 2, N, L)
    F[3:9, 2:12] = 0.0
    c = efm.collide_modes(p, F)
    z = F == 0.0
    assert np.all(c.Q[z] >= -1e-14 * np.abs(c.Qplus).max())
    assert c.Q[z].max() > 0.0


def test_forward_euler_positivity_and_entropy():
    """F + dt Q = F(1 - dt l) + dt Q+ >= 0 when dt max l <= 1; the entropy
    eta (section 4.2) is non-increasing up to the O(dt^2) forward-Euler term."""
    N, L = 16, 8.0
    p = efm.make_plan(N, 2, L, 8, R=R)
    F = _mix(3, 2, N, L) + 1e-8
    h2 = p.h ** 2
    eta_prev = None
    for step in range(30):
        c = efm.collide_modes(p, F)
        ell = efm.collision_frequency(p, F)
        dt = min(0.05, 1.0 / ell.max())
        Fn = F + dt * c.Q
        assert Fn.min() >= -1e-14 * Fn.max()
        eta = h2 * np.sum(F * np.log(F))
        if eta_prev is not None:
            bound = dt * dt * h2 * np.sum(c.Q ** 2 / F)
            assert eta <= eta_prev + bound
        eta_prev = eta
        F = np.maximum(Fn, 1e-300)


# --------------------------------------------------------------------------
# Accuracy: closed forms and the printed tables (section 4.2)
# --------------------------------------------------------------------------

def test_bkw_closed_forms_consistent():
    for d in (2, 3):
        N, L = 16, 8.0
        V2 = sum(x * x for x in synth.velocity_grid(N, d, L))
        for t in (0.0, 0.3, 2.0):
            assert np.abs(synth.bkw(d, t, N, L) - efm.bkw_f(d, t, V2)).max() < 1e-15
            dtau = 1e-5
            fd = (efm.bkw_f(d, t + dtau, V2) - efm.bkw_f(d, t - dtau, V2)) / (2 * dtau)
            assert np.abs(fd - efm.bkw_dfdt(d, t, V2)).max() < 1e-8 * np.abs(fd).max()


def test_bkw_collision_term_converges():
    """Q^sigma[I_N f(t0)] approaches df/dt of the BKW solution (exact for the
    continuous Maxwell operator) as N grows; the paper's argument (section
    3.3) gives order 2 asymptotically, pre-asymptotic rates are lower."""
    errs = []
    for N in (16, 32, 64):
        p = efm.make_plan(N, 2, T_PAPER, 8, R=R)
        V2 = sum(x * x for x in synth.velocity_grid(N, 2, T_PAPER))
        q = efm.collide_modes(p, efm.bkw_f(2, 0.5, V2)).Q
        g = efm.bkw_dfdt(2, 0.5, V2)
        errs.append(np.linalg.norm(q - g) / np.linalg.norm(g))
    assert errs[0] > errs[1] > errs[2]
    assert math.log2(errs[1] / errs[2]) > 1.4


def _rk3_errors(N, M):
    p = efm.make_plan(N, 2, T_PAPER, M, R=R)
    V2 = sum(x * x for x in synth.velocity_grid(N, 2, T_PAPER))
    F0 = synth.bkw(2, 0.0, N, T_PAPER)
    u = efm.ssprk3_step(lambda f: efm.collide_modes(p, f).Q, F0, 0.01)
    fe = efm.bkw_f(2, 0.01, V2)
    e = (u - fe).ravel(); f = fe.ravel()
    return (np.abs(e).sum() / np.abs(f).sum(), np.linalg.norm(e) / np.linalg.norm(f),
            np.abs(e).max() / np.abs(f).max())


@pytest.mark.parametrize("N", [16, 32, 64])
def test_table2_fast_algorithm_errors(golden, N):
    """Section 4.2, Table 2: l1 errors for M = 2, 3, 32, reproduced to the
    printed digits (this fixes T = (3 sqrt 2 + 1) R / 4, the even-N filter and
    the node placement)."""
    tab = golden("table2_fast_l1.txt")
    row = tab[tab[:, 0] == N][0]
    for col, M in ((1, 2), (2, 3), (3, 32)):
        l1 = _rk3_errors(N, M)[0]
        assert l1 == pytest.approx(row[col], rel=2e-4), (N, M, l1, row[col])


@pytest.mark.parametrize("N", [16, 32, 64])
def test_table1_bkw_errors(golden, N):
    """Section 4.2, Table 1 (printed to 3 digits)."""
    tab = golden("table1_bkw2d.txt")
    row = tab[tab[:, 0] == N][0]
    l1, l2, li = _rk3_errors(N, 32)
    assert l1 == pytest.approx(row[1], rel=6e-3)
    assert l2 == pytest.approx(row[2], rel=6e-3)
    assert li == pytest.approx(row[3], rel=6e-3)


def test_maxwellian_residual_decreases():
    """A resolved Maxwellian is an equilibrium of the continuous operator; the
    filter smears it (section 3.3), so ||Q||/||Q+|| is small and falls about
    4x per doubling of N."""
    r = []
    for N in (16, 32, 64):
        p = efm.make_plan(N, 2, T_PAPER, 8, R=R)
        V2 = sum(x * x for x in synth.velocity_grid(N, 2, T_PAPER))
        c = efm.collide_modes(p, np.exp(-V2 / 2) / (2 * math.pi))
        r.append(np.linalg.norm(c.Q) / np.linalg.norm(c.Qplus))
    assert r[2] < 0.05
    assert r[0] / r[1] > 2.8 and r[1] / r[2] > 2.8


def test_momentum_energy_not_conserved_but_converge():
    """Section 5: EFM does not conserve momentum or energy; the defects are
    non-zero and shrink with N (asserting exact conservation would be wrong)."""
    en = []
    for N in (16, 32, 64):
        p = efm.make_plan(N, 2, T_PAPER, 8, R=R)
        F = _mix(9, 2, N, T_PAPER)
        c = efm.collide_modes(p, F)
        m = efm.monitors(p, F, c.Q)
        en.append(abs(m["energy"]))
        assert abs(m["energy"]) > 1e-8
    assert en[0] > en[1] > en[2]


def test_time_integrators_on_a_linear_ode():
    """The oracle's forward Euler and SSP-RK3 (Shu-Osher form, the paper's
    integrator, section 4.1) on u' = lam u: one step multiplies u by the
    stability polynomial, 1 + z and 1 + z + z^2/2 + z^3/6 (z = lam dt), the
    latter being third order; a wrong stage weight changes the polynomial."""
    u = np.array([1.0, -2.0, 0.5])
    for lam, dt in ((-3.0, 0.01), (-0.7, 0.3), (1.3, 0.05)):
        z = lam * dt
        op = lambda v: lam * v   # noqa: E731
        assert np.allclose(efm.fe_step(op, u, dt), (1 + z) * u, rtol=1e-15, atol=0)
        assert np.allclose(efm.ssprk3_step(op, u, dt), (1 + z + z * z / 2 + z ** 3 / 6) * u,
                           rtol=1e-14, atol=0)


@pytest.mark.parametrize("d,N,M", [(2, 8, 4), (3, 6, 8)])
def test_dense_kernel_sum_equals_low_rank_double_sum(d, N, M):
    """collide_dense (numpy sum of eq. EFMk over a dense kernel-mode matrix)
    with the low-rank kernel written out densely equals the C double sum of
    eq. Qsk (two codes of the same definition)."""
    L = 8.0
    p = efm.make_plan(N, d, L, M, R=R)
    F = _mix(61 + N, d, N, L)
    q = efm.collide_dense(p.lr.matrix(), p.sigma, F, L)
    ref = efm.collide_modes(p, F)
    assert np.abs(q - ref.Q).max() <= 1e-13 * np.abs(ref.Qplus).max()

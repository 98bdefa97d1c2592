"""CPU pins of the oracle's non-separable 3D kernels (variable hard spheres
and 3D Maxwell molecules through radial quadrature), each against something
other than the oracle's own formula:

- gamma = 1 must give the hard-sphere kernel (sinc / J_1 closed forms pinned
  elsewhere) as the radial rule is refined;
- B(0, 0) has a closed form for every gamma:
  8 pi int_0^R int_0^R (p^2 + s^2)^a p s dp ds
  = 8 pi R^{2a+4} (2^{a+2} - 2) / (4 (a+1)(a+2)),  a = (gamma - 1)/2;
- the Hankel factor equals scipy's adaptive quadrature of its integral;
- Theorem 1 (mass, H-theorem) and the DVM brute force for the new kernel;
- the 3D Maxwell operator approaches the BKW time derivative as N grows.
"""
import math

import numpy as np
import pytest

import synth
from oracle import efm

R = 6.0


def test_gamma_one_reduces_to_hard_spheres():
    p = efm.make_plan(6, 3, 8.0, 8, kind=efm.KIND_VHS, gamma=1.0, n_radial=24)
    h = efm.make_plan(6, 3, 8.0, 8)
    A, B = p.lr.matrix(), h.lr.matrix()
    assert np.abs(A - B).max() <= 1e-12 * np.abs(B).max()


@pytest.mark.parametrize("gamma,nr", [(0.0, 16), (0.5, 96)])
def test_origin_value_closed_form(gamma, nr):
    kind = efm.KIND_MAXWELL if gamma == 0.0 else efm.KIND_VHS
    p = efm.make_plan(4, 3, 8.0, 8, kind=kind, gamma=gamma, n_radial=nr)
    a = 0.5 * (gamma - 1.0)
    closed = 8 * math.pi * R ** (2 * a + 4) * (2 ** (a + 2) - 2) / (4 * (a + 1) * (a + 2))
    k0 = np.where((np.array(efm.mode_grid(4, 3)) == 0).all(0))[0][0]
    got = p.lr.matrix()[k0, k0]
    assert got == pytest.approx(closed, rel=5e-12)


@pytest.mark.parametrize("rho,a,q", [(0.01, -0.5, 3.7), (1.3, -0.25, 11.2), (0.2, -0.25, 0.0),
                                     (4.0, -0.5, 20.0), (0.003, -0.25, 17.0), (2.5, 0.0, 5.5)])
def test_hankel_factor_against_adaptive_quadrature(rho, a, q):
    from scipy.integrate import quad
    from scipy.special import j0
    ref = 4 * math.pi * quad(lambda r: (rho * rho + r * r) ** a * j0(q * r) * r, 0, R,
                             limit=1000, epsabs=1e-15, epsrel=1e-13,
                             points=[rho, 2 * rho, 8 * rho])[0]
    got = efm.hankel_disk(np.array([q]), rho, a, R)[0]
    assert abs(got - ref) <= 2e-12 * max(abs(ref), 4 * math.pi * R)


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_theorem1_for_nonseparable_kernels(gamma):
    N, L = 8, 8.0
    kind = efm.KIND_MAXWELL if gamma == 0.0 else efm.KIND_VHS
    p = efm.make_plan(N, 3, L, 8, kind=kind, gamma=gamma, n_radial=4)
    F = synth.sample_mixture(synth.mixture_anisotropic(77, 3), N, L)
    c = efm.collide_modes(p, F)
    assert abs(c.Q.sum()) <= 1e-13 * np.abs(c.Q).sum()
    assert np.sum(c.Q * np.log(F)) <= 0.0
    assert c.imag_max <= 1e-13 * np.abs(c.Qplus).max()


def test_dvm_brute_force_for_vhs():
    p = efm.make_plan(4, 3, 8.0, 2, kind=efm.KIND_VHS, gamma=0.5, n_radial=2)
    A = efm.dvm_tensor(p)
    assert A.min() >= -1e-14 * A.max()
    F = synth.sample_mixture(synth.mixture_anisotropic(3, 3), 4, 8.0)
    q_dvm = efm.collide_dvm(A, F)
    q = efm.collide_modes(p, F).Q
    assert np.abs(q_dvm - q).max() <= 1e-12 * np.abs(q).max()


def test_maxwell_3d_approaches_bkw_derivative():
    """Pre-asymptotic but monotone: the sampled relative error of Q against
    df/dt of the 3D BKW solution (section 4.2, Example 4) at t = 0.5 falls
    from N = 24 to N = 32."""
    T = efm.default_box(R)
    errs = []
    for N in (24, 32):
        p = efm.make_plan(N, 3, T, 8, kind=efm.KIND_MAXWELL, R=R, n_radial=8)
        V2 = sum(x * x for x in synth.velocity_grid(N, 3, T))
        F = efm.bkw_f(3, 0.5, V2)
        g = efm.bkw_dfdt(3, 0.5, V2).ravel()
        cand = np.nonzero(V2.ravel() < 16.0)[0]
        idx = np.random.default_rng(0).choice(cand, 150, replace=False)
        q = efm.collide_points(p, F, idx)[0]
        errs.append(np.linalg.norm(q - g[idx]) / np.linalg.norm(g[idx]))
    assert errs[1] < 0.85 * errs[0]


def test_sparse_support_plan_equals_full_plan():
    """A plan restricted to the modes where the input's spectrum lives (a
    real trigonometric polynomial) gives the same point form of the fast
    algorithm as the full plan (section 4.1, eq. fastAlg: every sum over
    modes k carries Fh_k, which vanishes off the support) and the same
    operator as the double sum of eq. Qsk; an input with spectrum off the
    support is refused."""
    N, L, R = 12, 8.0, 6.0
    F, modes = synth.trig_polynomial(5, N, 3, L, n_waves=10)
    assert modes.shape == (3, 21)
    kw = dict(kind=efm.KIND_VHS, R=R, gamma=0.5, n_radial=3)
    full = efm.make_plan(N, 3, L, 8, **kw)
    sp = efm.make_plan(N, 3, L, 8, modes=modes, **kw)
    idx = np.arange(N ** 3)
    a = efm.collide_points(full, F, idx)
    b = efm.collide_points(sp, F, idx)
    ref = efm.collide_modes(full, F)
    scale = np.abs(ref.Qplus).max()
    assert np.abs(a[0] - b[0]).max() <= 1e-13 * scale
    assert np.abs(b[0] - ref.Q.ravel()).max() <= 1e-13 * scale
    assert np.abs(b[1] - ref.Qplus.ravel()).max() <= 1e-13 * scale
    # the polynomial's spectrum: exactly the listed modes (to roundoff)
    Fh = efm.dft(F, L)
    on = np.zeros(Fh.shape, bool)
    on[tuple(m % N for m in modes)] = True
    assert np.abs(Fh[~on]).max() <= 1e-15 * np.abs(Fh).max()
    with pytest.raises(ValueError):
        efm.collide_points(sp, synth.sample_mixture(synth.mixture_two_gaussians(1, 3), N, L), idx[:4])

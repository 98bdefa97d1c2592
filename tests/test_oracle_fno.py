"""CPU checks of the surrogate's FP64 reference network (oracle/fno.py).

The surrogate is not in the paper, so these pin the reference against
independent evaluations of the definitions it writes out: an explicit
plane-wave sum for the spectral convolution, the pointwise limit, and the
adjointness of the truncated transform pair used by the backward pass."""
import math

import numpy as np

from oracle import fno


def test_spectral_conv_single_mode_is_a_plane_wave():
    N, K, C = 8, 2, 2
    rng = np.random.default_rng(0)
    u = rng.standard_normal((C, N, N, N))
    NM = 4 * K ** 3
    R = np.zeros((NM, C, C), dtype=complex)
    kx, ky, kz = fno.kept_indices(N, K)
    m = 5                                   # mode (mx, my, mz) in (kz fastest, then ky)
    mx, my, mz = m // (2 * K * K), (m // K) % (2 * K), m % K
    R[m, 1, 0] = 0.3 - 0.7j
    s = fno.spectral(u, R, N, K)
    # explicit: Uh = sum_r u[1](r) e^{-2 pi i k.r/N}; s[0](r) = Re(R Uh e^{+2 pi i k.r/N}) / N^3
    k = np.array([kx[mx], ky[my], kz[mz]])
    r = np.stack(np.meshgrid(*([np.arange(N)] * 3), indexing="ij"), axis=-1)
    ph = np.exp(2j * math.pi * (r @ k) / N)
    uh = np.sum(u[1] * np.conj(ph))
    ref = np.real(R[m, 1, 0] * uh * ph) / N ** 3
    assert np.abs(s[0] - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(s[1]).max() < 1e-12


def test_without_spectral_weights_the_network_is_pointwise():
    N, K, C, L = 8, 2, 3, 2
    rng = np.random.default_rng(1)
    p = rng.standard_normal(fno.n_params(N, K, C, L)) * 0.3
    for name, o, size in fno.param_blocks(N, K, C, L):
        if name.startswith("R"):
            p[o:o + size] = 0.0
    P = fno.unpack(p, N, K, C, L)
    x = rng.standard_normal((2, N ** 3))
    y = fno.forward(p, x, N, K, C, L)
    for b in range(2):
        u = P["Wl"][:, None] * x[b][None] + P["bl"][:, None]
        h = P["W"][0] @ u + P["b"][0][:, None]
        u = fno.gelu(h)
        h = P["W"][1] @ u + P["b"][1][:, None]
        ref = P["Wp"] @ h + P["bp"]
        assert np.abs(y[b] - ref).max() < 1e-12


def test_truncated_transform_pair_is_adjoint():
    """<S_R(u), w> = <u, S_R^*(w)> with S_R^* the same transforms with
    conj(R) transposed -- the identity the library's backward pass uses."""
    N, K, C = 8, 2, 3
    rng = np.random.default_rng(2)
    NM = 4 * K ** 3
    R = rng.standard_normal((NM, C, C)) + 1j * rng.standard_normal((NM, C, C))
    u = rng.standard_normal((C, N, N, N))
    w = rng.standard_normal((C, N, N, N))
    lhs = np.sum(fno.spectral(u, R, N, K) * w)
    Radj = np.conj(np.transpose(R, (0, 2, 1)))
    # the adjoint maps w through DFT (e^{-i}), mixes with conj(R)^T, inverse DFT, real part
    rhs = np.sum(u * fno.spectral(w, Radj, N, K))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_fd_gradient_matches_linear_layer_closed_form():
    """For the projection bias the gradient is closed-form: dL/dbp =
    mean_b 2 sum (y - t) / sum t^2."""
    N, K, C, L = 8, 2, 2, 1
    rng = np.random.default_rng(3)
    p = rng.standard_normal(fno.n_params(N, K, C, L)) * 0.2
    x = rng.standard_normal((2, N ** 3))
    t = rng.standard_normal((2, N ** 3))
    y = fno.forward(p, x, N, K, C, L)
    ref = np.mean(2 * np.sum(y - t, axis=1) / np.sum(t ** 2, axis=1))
    g = fno.fd_grad(p, x, t, N, K, C, L, [p.size - 1])
    assert abs(g[0] - ref) < 1e-7 * max(1.0, abs(ref))


def test_mass_projection_is_the_least_norm_correction():
    """The projection zeroes the mass, is idempotent, equals Q minus the
    minimum-norm correction with Q's mass (scipy's least squares), and never
    increases the distance to a target of zero mass."""
    from scipy.linalg import lstsq
    N = 6
    rng = np.random.default_rng(4)
    Q = rng.standard_normal((N, N, N)) + 0.3
    P = fno.mass_projection(Q)
    assert abs(P.sum()) < 1e-12 * np.abs(Q).sum()
    assert np.abs(fno.mass_projection(P) - P).max() < 1e-15
    A = np.ones((1, N ** 3))
    c = lstsq(A, A @ Q.ravel())[0]
    assert np.abs((Q.ravel() - c) - P.ravel()).max() < 1e-12 * np.abs(Q).max()
    for _ in range(5):
        target = fno.mass_projection(rng.standard_normal((N, N, N)))
        assert np.linalg.norm(P - target) <= np.linalg.norm(Q - target) + 1e-12

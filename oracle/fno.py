"""FP64 CPU reference of the learned surrogate (a Fourier neural operator).

TEST INFRASTRUCTURE ONLY.  The surrogate is not part of the paper; this module
is the plain definition of the network the library trains, written with numpy
FFTs, so that the library's FP32 forward pass and its hand-written backward
pass can be checked (forward values, and gradients against central
differences of this forward pass).

Network (n = N^3 grid points, C channels, kept modes kx, ky in [-K, K),
kz in [0, K)):
    u0[c] = Wl[c] x + bl[c]
    h_l   = W_l u + b_l + Re IDFT(scatter(R_l . DFT(u)|kept))
            (forward DFT unnormalised, inverse DFT normalised by 1/N^3)
    u     = GELU(h_l) for l < L-1, u = h_{L-1} for the last layer
    y     = sum_c Wp[c] u[c] + bp
Flat parameter layout: Wl[C], bl[C], per layer W[C][C] (out, in), b[C],
R[modes][C][C] (in, out) as (re, im) pairs, then Wp[C], bp.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def kept_indices(N, K):
    k = np.concatenate([np.arange(K), np.arange(N - K, N)])
    return k, k, np.arange(K)


def unpack(p, N, K, C, L):
    p = np.asarray(p, dtype=np.float64)
    NM = 4 * K ** 3
    o = 0
    out = {}
    out["Wl"] = p[o:o + C]; o += C
    out["bl"] = p[o:o + C]; o += C
    out["W"], out["b"], out["R"] = [], [], []
    for _ in range(L):
        out["W"].append(p[o:o + C * C].reshape(C, C)); o += C * C
        out["b"].append(p[o:o + C]); o += C
        r = p[o:o + 2 * NM * C * C]; o += 2 * NM * C * C
        out["R"].append((r[0::2] + 1j * r[1::2]).reshape(NM, C, C))
    out["Wp"] = p[o:o + C]; o += C
    out["bp"] = p[o]; o += 1
    assert o == p.size, (o, p.size)
    return out


def n_params(N, K, C, L):
    return 2 * C + L * (C * C + C + 2 * 4 * K ** 3 * C * C) + C + 1


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def spectral(u, R, N, K):
    """u: [C, N, N, N] real; R: [NM, C, C]; returns [C, N, N, N] real.
    Mode order: (mx over kx, my over ky, kz) with kz fastest, then ky."""
    kx, ky, kz = kept_indices(N, K)
    C = u.shape[0]
    U = np.fft.fftn(u, axes=(1, 2, 3))                      # unnormalised forward
    Uh = U[:, kx][:, :, ky][:, :, :, kz]                    # [C, 2K, 2K, K]
    Uh = Uh.reshape(C, -1).T                                # [NM, C]
    V = np.einsum("mio,mi->mo", R, Uh)                      # [NM, C]
    S = np.zeros((C, N, N, N), dtype=np.complex128)
    Vb = V.T.reshape(C, 2 * K, 2 * K, K)
    S[np.ix_(np.arange(C), kx, ky, kz)] = Vb
    return np.real(np.fft.ifftn(S, axes=(1, 2, 3)))           # normalised inverse


def forward(p, x, N, K, C, L):
    """x: [B, n] -> y: [B, n]."""
    P = unpack(p, N, K, C, L)
    B = x.shape[0]
    ys = []
    for b in range(B):
        xb = np.asarray(x[b], dtype=np.float64).reshape(N, N, N)
        u = P["Wl"][:, None, None, None] * xb[None] + P["bl"][:, None, None, None]
        for l in range(L):
            s = spectral(u, P["R"][l], N, K)
            h = np.einsum("oi,ixyz->oxyz", P["W"][l], u) + P["b"][l][:, None, None, None] + s
            u = gelu(h) if l + 1 < L else h
        y = np.einsum("c,cxyz->xyz", P["Wp"], u) + P["bp"]
        ys.append(y.ravel())
    return np.stack(ys)


def loss(p, x, t, N, K, C, L):
    """Mean over samples of sum (y - t)^2 / sum t^2."""
    y = forward(p, x, N, K, C, L)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean(np.sum((y - t) ** 2, axis=1) / (np.sum(t ** 2, axis=1) + 1e-30)))


def fd_grad(p, x, t, N, K, C, L, idx, eps=1e-6):
    """Central differences of the loss with respect to the parameters idx."""
    p = np.asarray(p, dtype=np.float64).copy()
    g = np.empty(len(idx))
    for j, i in enumerate(idx):
        h = eps * max(1.0, abs(p[i]))
        old = p[i]
        p[i] = old + h
        lp = loss(p, x, t, N, K, C, L)
        p[i] = old - h
        lm = loss(p, x, t, N, K, C, L)
        p[i] = old
        g[j] = (lp - lm) / (2 * h)
    return g


def param_blocks(N, K, C, L):
    """(name, offset, size) of every parameter block in the flat layout."""
    NM = 4 * K ** 3
    o, out = 0, []
    for name, size in [("Wl", C), ("bl", C)]:
        out.append((name, o, size)); o += size
    for l in range(L):
        for name, size in [(f"W{l}", C * C), (f"b{l}", C), (f"R{l}", 2 * NM * C * C)]:
            out.append((name, o, size)); o += size
    for name, size in [("Wp", C), ("bp", 1)]:
        out.append((name, o, size)); o += size
    return out


def mass_projection(Q):
    """Q - mean(Q): the orthogonal projection of Q onto grid functions whose
    discrete mass vanishes."""
    Q = np.asarray(Q, dtype=np.float64)
    return Q - Q.mean()

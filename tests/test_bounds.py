"""The stated reduced-precision bounds (paper_1704_07369_amd.bounds) against
a plain FP32 model of the fast algorithm on the CPU: the oracle's tables
rounded to FP32, single-precision FFTs (scipy), FP64 sums over the terms, as
the FP32 path computes (section 4.1, eq. fastAlg).  The worst-case bound
must hold with room to spare; a model that drops precision further (FP16
spectra) must break it, so the test can fail."""
import numpy as np
import pytest
import scipy.fft as sfft

import synth
from oracle import efm
from paper_1704_07369_amd import bounds


def fp32_model(plan, F):
    N, d = plan.N, plan.d
    shp = (N,) * d
    n = N ** d
    # library normalisation: c_t = IDFT_unnormalised(gamma_t DFT_unnormalised(F)),
    # gamma_t = (c_t sigma U_t + i sigma V_t) / n; the phases of the grid offset
    # cancel in every product
    lr, sig = plan.lr, plan.sigma
    Fh = sfft.fftn(F.astype(np.complex64))
    qp = np.zeros(shp)
    for t in range(len(lr.c)):
        g = ((lr.c[t] * sig * lr.U[t] + 1j * sig * lr.V[t]) / n).reshape(shp).astype(np.complex64)
        c = sfft.ifftn(g * Fh) * n
        qp += c.real.astype(np.float64) * c.imag.astype(np.float64)
    D = (sig * sig * lr.diagonal() / n).reshape(shp).astype(np.complex64)
    ell = (sfft.ifftn(D * Fh) * n).real.astype(np.float64)
    return qp - F * ell


@pytest.mark.parametrize("N,d,M", [(16, 3, 32), (32, 2, 16)])
def test_fp32_model_within_stated_bound(N, d, M):
    L = 8.0
    p = efm.make_plan(N, d, L, M, R=6.0)
    for seed in range(2):
        F = synth.sample_mixture(synth.mixture_anisotropic(40 + seed, d), N, L)
        ref = efm.collide_modes(p, F)
        den = np.linalg.norm(ref.Qplus)
        r = np.linalg.norm(ref.Qminus) / den
        err = np.linalg.norm(fp32_model(p, F) - ref.Q) / den
        tol = bounds.fp32_bound(N, d, r)
        assert err <= tol, (err, tol)
        assert err >= 1e-9          # it is an FP32 computation


def test_fp16_spectra_break_the_fp32_bound():
    N, d, M, L = 16, 3, 32, 8.0
    p = efm.make_plan(N, d, L, M, R=6.0)
    F = synth.sample_mixture(synth.mixture_anisotropic(40, d), N, L)
    ref = efm.collide_modes(p, F)
    den = np.linalg.norm(ref.Qplus)
    r = np.linalg.norm(ref.Qminus) / den
    # spectra rounded to FP16 significands (11 bits) before each inverse transform
    lr, sig, n, shp = p.lr, p.sigma, N ** d, (N,) * d
    Fh = sfft.fftn(F)
    Fh = (Fh.real.astype(np.float16).astype(np.float64)
          + 1j * Fh.imag.astype(np.float16).astype(np.float64))
    qp = np.zeros(shp)
    for t in range(len(lr.c)):
        g = ((lr.c[t] * sig * lr.U[t] + 1j * sig * lr.V[t]) / n).reshape(shp)
        c = sfft.ifftn(g * Fh) * n
        qp += c.real * c.imag
    ell = (sfft.ifftn((sig * sig * lr.diagonal() / n).reshape(shp) * Fh) * n).real
    err = np.linalg.norm(qp - F * ell - ref.Q) / den
    assert err > bounds.fp32_bound(N, d, r)

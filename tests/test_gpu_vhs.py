"""GPU parity of the non-separable 3D kernels (3D Maxwell molecules and
variable hard spheres, M' = M n_radial radial products) and of the 64^3
grids, against the CPU oracle.

Bars: FP64 1e-12 of the gain (full grid at 16^3, sampled points above),
FP32 transforms 1e-5, split-BF16 x pass 5e-4 (the derivations are those of
the separable kernels: the radial products change the number of terms, not
the rounding of each transform).  At 64^3 the oracle's tables cost
O(n M' quadrature), so those cases keep M' small.
"""
import numpy as np
import pytest

import synth
from oracle import efm
from tests.gpu_util import rel_err, say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R, L = 6.0, 8.0
TOL = {0: 1e-12, 1: 1e-5, 2: 5e-4}


def plans(N, M, gamma, nr):
    if gamma == 1.0:
        return E.Plan(N, 3, L, M, R=R), efm.make_plan(N, 3, L, M, R=R)
    kind = E.EC_KERNEL_MAXWELL if gamma == 0.0 else E.EC_KERNEL_VHS
    okind = efm.KIND_MAXWELL if gamma == 0.0 else efm.KIND_VHS
    return (E.Plan(N, 3, L, M, kind=kind, R=R, gamma=gamma, n_radial=nr),
            efm.make_plan(N, 3, L, M, kind=okind, R=R, gamma=gamma, n_radial=nr))


def run(p, cells, precision, mode=None, split=0):
    import torch
    b = E.Batch([p], [len(cells)], precision)
    if mode is not None:
        b.set_schedule(0, mode, 0, split)
    say(f"  schedule {b.get_schedule(0)}")
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    return E.unpack(b, Q.cpu().numpy())


@pytest.mark.parametrize("gamma,prec,mode,split", [
    (0.0, 0, 2, 1), (0.0, 0, 1, 0), (0.5, 0, 2, 2), (0.5, 1, 2, 1), (0.5, 2, 1, 0),
])
def test_nonseparable_16_full_grid(gamma, prec, mode, split):
    say(f"case non-separable 16^3 gamma={gamma} precision={prec} mode={mode} split={split}")
    N, M, nr = 16, 8, 4
    p, op = plans(N, M, gamma, nr)
    assert p.terms() == M * nr
    cells = [synth.sample_mixture(synth.mixture_anisotropic(9400 + i, 3), N, L) for i in range(3)]
    out = run(p, cells, prec, mode, split)
    for c in range(3):
        ref = efm.collide_modes(op, cells[c])
        err = rel_err(out[c], ref.Q, ref.Qplus)
        say(f"  cell {c}: rel err {err:.3e}")
        assert err <= TOL[prec]
        if prec == 0:
            assert abs(out[c].sum()) <= 1e-13 * np.abs(out[c]).sum()


def test_vhs_32_sampled():
    say("case VHS 32^3 sampled")
    N, M, nr = 32, 8, 4
    p, op = plans(N, M, 0.5, nr)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(9500 + i, 3), N, L) for i in range(2)]
    out = run(p, cells, 0)
    rng = np.random.default_rng(9)
    for c in range(2):
        idx = rng.choice(N ** 3, 40, replace=False)
        q, qp, _, _ = efm.collide_points(op, cells[c], idx)
        err = np.abs(out[c].ravel()[idx] - q).max() / np.abs(qp).max()
        say(f"  cell {c}: max rel err {err:.3e}")
        assert err <= 1e-12


@pytest.mark.parametrize("gamma,M,nr", [(1.0, 4, 1), (0.5, 2, 2)])
def test_64_sampled_all_precisions(gamma, M, nr):
    say(f"case 64^3 gamma={gamma} M={M} n_radial={nr}")
    N = 64
    p, op = plans(N, M, gamma, nr)
    cells = [synth.sample_mixture(synth.mixture_two_gaussians(9600 + i, 3), N, L) for i in range(2)]
    # half of the samples where F peaks, so that max |Q+| over the samples is
    # the gain's scale (random points alone can miss a narrow component)
    rng = np.random.default_rng(64)
    idx = [np.unique(np.concatenate([np.argsort(cells[c].ravel())[-16:],
                                     rng.choice(N ** 3, 16, replace=False)])) for c in range(2)]
    refs = [efm.collide_points(op, cells[c], idx[c]) for c in range(2)]
    for prec in (0, 1, 2):
        out = run(p, cells, prec)
        for c in range(2):
            q, qp = refs[c][0], refs[c][1]
            err = np.abs(out[c].ravel()[idx[c]] - q).max() / np.abs(qp).max()
            say(f"  precision {prec} cell {c}: max rel err {err:.3e}")
            assert err <= TOL[prec]

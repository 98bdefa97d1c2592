"""GPU parity of the non-separable 3D kernels (3D Maxwell molecules and
variable hard spheres, M' = M n_radial radial products) and of the 64^3
grids, against the CPU oracle.

Bars (paper_1704_07369_amd.bounds, stated a priori): FP64 1e-12 of the gain
(full grid at 16^3 and at the 64^3 sweep plan, sampled points elsewhere);
FP32 transforms and the split-BF16 x pass at their per-size bounds (the
radial products change the number of terms, not the rounding of each
transform).  The oracle's tables on a full 64^3 grid cost O(n M')
quadratures, so the Gaussian-mixture cases at 64^3 keep M' small; the
precision-sweep plan itself (M' = 512) is checked on inputs whose spectrum
lives on a few modes, where the oracle needs its tables there only.
"""
import numpy as np
import pytest

import synth
from oracle import efm
from paper_1704_07369_amd import bounds
from tests.gpu_util import rel_err, say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R, L = 6.0, 8.0


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
        tol = bounds.bound(prec, N, 3, np.linalg.norm(ref.Qminus) / np.linalg.norm(ref.Qplus))
        say(f"  cell {c}: rel err {err:.3e} (bound {tol:.3e})")
        assert err <= tol
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
            q, qp, qm = refs[c][0], refs[c][1], refs[c][2]
            err = np.abs(out[c].ravel()[idx[c]] - q).max() / np.abs(qp).max()
            tol = bounds.bound(prec, N, 3, np.abs(qm).max() / np.abs(qp).max())
            say(f"  precision {prec} cell {c}: max rel err {err:.3e} (bound {tol:.3e})")
            assert err <= tol


# the precision-sweep workload's plan and schedules: 64^3, variable hard
# spheres gamma = 0.5, M = 64 directions x 8 radial nodes (512 products);
# FP64 in two-pass passes of 23 cells (the sweep's measured schedule)
C4 = dict(N=64, M=64, nr=8, gamma=0.5)


def _points_chunked(op, F, chunk=16384):
    n = F.size
    q = np.empty(n); qp = np.empty(n); qm = np.empty(n)
    for i in range(0, n, chunk):
        idx = np.arange(i, min(n, i + chunk))
        q[idx], qp[idx], qm[idx], _ = efm.collide_points(op, F, idx)
    shp = F.shape
    return q.reshape(shp), qp.reshape(shp), qm.reshape(shp)


def test_sweep_plan_full_grid_sparse_spectrum():
    """The 64^3 sweep plan (513 transforms per evaluation) on the full grid of
    two cells (the first cell of each two-pass pass of 23) against the
    oracle's point form of the fast algorithm (section 4.1, eq. fastAlg),
    FP64, FP32 and split-BF16.  The inputs are real trigonometric
    polynomials (background 1, 12 random waves, F in [0.5, 1.5]) whose
    spectrum lives on 25 known modes, so the oracle's quadrature tables are
    needed on those modes only; the GPU transforms the whole grid."""
    import torch
    N, M, nr, gam = C4["N"], C4["M"], C4["nr"], C4["gamma"]
    say(f"case sweep plan 64^3 M={M} x n_radial={nr} gamma={gam}, full grid, sparse spectra")
    p = E.Plan(N, 3, L, M, kind=E.EC_KERNEL_VHS, R=R, gamma=gam, n_radial=nr)
    assert p.terms() == M * nr
    ncell = 24
    inputs = [synth.trig_polynomial(7001 + c, N, 3, L) for c in range(ncell)]
    cells = [F for F, _ in inputs]
    check = [0, 23]
    refs = {}
    for c in check:
        op = efm.make_plan(N, 3, L, M, kind=efm.KIND_VHS, R=R, gamma=gam, n_radial=nr,
                           modes=inputs[c][1])
        refs[c] = _points_chunked(op, cells[c])
        say(f"  oracle cell {c} done")
    for prec, mode, chunk in ((0, E.EC_SCHED_TWO_PASS, 23), (1, None, 0), (2, None, 0)):
        b = E.Batch([p], [ncell], prec)
        if mode is not None:
            b.set_schedule(0, mode, chunk, 0)
        say(f"  precision {prec} schedule {b.get_schedule(0)}")
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.collide(f, Q)
        torch.cuda.synchronize()
        out = E.unpack(b, Q.cpu().numpy())
        b.close()
        for c in check:
            q, qp, qm = refs[c]
            err = rel_err(out[c], q, qp)
            tol = bounds.bound(prec, N, 3, np.linalg.norm(qm) / np.linalg.norm(qp))
            say(f"  precision {prec} cell {c}: rel err {err:.3e} (bound {tol:.3e})")
            assert err <= tol


def test_64_two_pass_euler_step_in_place():
    """The 64^3 slab pass's in-place forward-Euler update (F + dt Q written
    over F by the pass that computes Q) over a full pass of 23 cells and a
    tail pass of 2, FP64 and FP32: equal to F + dt Q from a separate collide
    of the same cells up to the rounding of the final update."""
    import torch
    say("case 64^3 two-pass Euler step in place, 25 cells in passes of 23")
    p = E.Plan(64, 3, L, 2, kind=E.EC_KERNEL_VHS, R=R, gamma=0.5, n_radial=2)
    cells = [synth.sample_mixture(synth.mixture_two_gaussians(9700 + i, 3), 64, L)
             for i in range(25)]
    dt = 0.01
    for prec in (0, 1):
        b = E.Batch([p], [len(cells)], prec)
        b.set_schedule(0, E.EC_SCHED_TWO_PASS, 23, 0)
        assert tuple(b.get_schedule(0))[:2] == (E.EC_SCHED_TWO_PASS, 23)
        f = to_dev(E.pack(b, cells))
        Q = torch.zeros_like(f)
        b.collide(f, Q)
        want = f + dt * Q
        b.step(f, dt, 1)
        torch.cuda.synchronize()
        err = ((f - want).abs().max() / want.abs().max()).item()
        say(f"  precision {prec}: max |step - (F + dt Q)| / max F = {err:.3e}")
        assert err <= 1e-14
        b.close()


def test_64_degenerate_cells():
    """Degenerate cells through the 64^3 passes (VHS gamma = 0.5, M' = 4, FP64
    and FP32): F = 0 gives Q = 0 exactly; a single-point spike stays finite;
    a mixture with a zeroed block matches the oracle on sampled points, half of
    them inside the block, where Q = Q+ >= 0 (the loss F l vanishes there;
    Theorem 1)."""
    say("case 64^3 degenerate cells")
    N = 64
    p, op = plans(N, 2, 0.5, 2)
    zero = np.zeros((N, N, N))
    spike = np.zeros((N, N, N))
    spike[N // 2, N // 2 + 3, N // 2 - 5] = 1.0
    holey = synth.sample_mixture(synth.mixture_two_gaussians(9800, 3), N, L)
    holey[24:36, 28:40, 20:44] = 0.0
    rng = np.random.default_rng(98)
    hole = np.ravel_multi_index(np.nonzero(holey == 0.0), holey.shape)
    idx = np.unique(np.concatenate([rng.choice(hole, 16, replace=False),
                                    np.argsort(holey.ravel())[-8:],
                                    rng.choice(N ** 3, 8, replace=False)]))
    q, qp, qm, _ = efm.collide_points(op, holey, idx)
    inside = holey.ravel()[idx] == 0.0
    assert inside.sum() >= 16 and np.abs(qm[inside]).max() == 0.0
    for prec in (0, 1):
        out = run(p, [zero, holey, spike], prec)
        assert np.all(out[0] == 0.0)
        assert np.all(np.isfinite(out[2]))
        err = np.abs(out[1].ravel()[idx] - q).max() / np.abs(qp).max()
        tol = bounds.bound(prec, N, 3, np.abs(qm).max() / np.abs(qp).max())
        low = out[1].ravel()[idx][inside].min() / np.abs(qp).max()
        say(f"  precision {prec}: max rel err {err:.3e} (bound {tol:.3e}), min Q in the hole "
            f"{low:.3e} of max Q+")
        assert err <= tol
        assert low >= -tol

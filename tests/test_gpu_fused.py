"""GPU parity of the fused schedule (every term's inverse transform on chip,
x axis split into P residue classes) against the CPU oracle, and against the
two-pass schedule on the same inputs.

Bars as in test_gpu_collide: FP64 1e-12 of the gain's norm (full grid at
16^3, sampled points at 24^3 and 32^3), FP32 transforms at their stated
per-size bound.  Cell counts
that are not multiples of 8 exercise the XCD-ordered block mapping, chunk
sizes below the cell count the ragged last pass.  N = 32 runs the column
form of the kernel (splits 2 and 4), N = 16 and 24 the LDS-volume form."""
import numpy as np
import pytest

import synth
from oracle import efm
from tests.gpu_util import bound_full, bound_pts, rel_err, say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R, L, M = 6.0, 8.0, 32

_plans = {}


def oplan(N):
    if N not in _plans:
        _plans[N] = efm.make_plan(N, 3, L, M, R=R)
    return _plans[N]


def run(N, cells, precision, mode, chunk, split):
    import torch
    p = E.Plan(N, 3, L, M, R=R)
    b = E.Batch([p], [len(cells)], precision)
    b.set_schedule(0, mode, chunk, split)
    say(f"  schedule {b.get_schedule(0)}")
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    return E.unpack(b, Q.cpu().numpy())


@pytest.mark.parametrize("N,prec,split,chunk,ncell", [
    (16, 0, 1, 0, 9), (16, 0, 2, 4, 5), (16, 1, 1, 0, 3), (16, 1, 2, 2, 3),
    (24, 0, 2, 2, 3), (24, 0, 3, 0, 3), (24, 1, 2, 0, 2), (24, 1, 3, 0, 2),
    (32, 0, 2, 0, 3), (32, 0, 2, 4, 9), (32, 0, 4, 2, 3), (32, 1, 2, 0, 2), (32, 1, 4, 0, 2),
    (32, 1, 2, 3, 7),
])
def test_fused_parity(N, prec, split, chunk, ncell):
    say(f"case fused N={N} precision={prec} split={split} chunk={chunk} cells={ncell}")
    cells = [synth.sample_mixture(synth.mixture_anisotropic(7100 + N + i, 3), N, L)
             for i in range(ncell)]
    out = run(N, cells, prec, E.EC_SCHED_FUSED, chunk, split)
    op = oplan(N)
    rng = np.random.default_rng(N + split)
    for c in range(ncell):
        assert np.all(np.isfinite(out[c]))
        if N == 16:
            ref = efm.collide_modes(op, cells[c])
            err = rel_err(out[c], ref.Q, ref.Qplus)
            tol = bound_full(prec, N, 3, ref)
        else:
            # the points where F peaks are among the samples, so that max |Q+|
            # over the samples is the gain's scale (random points alone can
            # miss a narrow component by a factor of 40)
            idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-12:],
                                            rng.choice(N ** 3, 40, replace=False)]))
            q, qp, qm, _ = efm.collide_points(op, cells[c], idx)
            err = np.abs(out[c].ravel()[idx] - q).max() / np.abs(qp).max()
            tol = bound_pts(prec, N, 3, qp, qm)
        say(f"  cell {c}: rel err {err:.3e} (bound {tol:.2e})")
        assert err <= tol


@pytest.mark.parametrize("N,split", [(24, 3), (32, 2), (32, 4)])
def test_fused_matches_two_pass_everywhere(N, split):
    """Full-grid agreement with the two-pass schedule (FP64, 11 cells)."""
    say(f"case fused vs two-pass N={N} split={split}")
    cells = [synth.sample_mixture(synth.mixture_anisotropic(7300 + i, 3), N, L) for i in range(11)]
    a = run(N, cells, 0, E.EC_SCHED_FUSED, 0, split)
    b = run(N, cells, 0, E.EC_SCHED_TWO_PASS, 0, 0)
    for c in range(11):
        d = np.linalg.norm(a[c] - b[c]) / np.linalg.norm(b[c])
        say(f"  cell {c}: |fused - two-pass| / |Q| = {d:.3e}")
        assert d <= 1e-12


@pytest.mark.parametrize("N", [16, 32])
def test_fused_step_in_place(N):
    """ec_step (Q written over f) under the fused schedule equals the two-pass
    schedule's step."""
    import torch
    say(f"case fused step in place N={N}")
    n = 6
    cells = [synth.sample_mixture(synth.mixture_anisotropic(7400 + i, 3), N, L) for i in range(n)]
    outs = []
    for mode in (E.EC_SCHED_FUSED, E.EC_SCHED_TWO_PASS):
        p = E.Plan(N, 3, L, M, R=R)
        b = E.Batch([p], [n])
        b.set_schedule(0, mode, 0, 0)
        f = to_dev(E.pack(b, cells))
        mon = torch.zeros(3 * n * 2, dtype=torch.float64, device="cuda")
        b.step(f, 0.01, 3, mon)
        torch.cuda.synchronize()
        outs.append((f.cpu().numpy(), mon.cpu().numpy()))
    assert np.abs(outs[0][0] - outs[1][0]).max() <= 1e-13 * np.abs(outs[1][0]).max()
    assert np.allclose(outs[0][1], outs[1][1], rtol=1e-12, atol=0)


@pytest.mark.parametrize("N,prec", [(24, 0), (24, 1), (32, 0), (32, 1)])
def test_forward_kernel_paths(N, prec):
    """The fused schedule's forward transform takes one workgroup per cell
    (k_fwd3) from 96 cells at 24^3 and 64 at 32^3, the slab pass and the
    in-place x pass below that.  The same cells in a batch of 128 and in a
    batch of 3 (fused, default split): both against the oracle on sampled
    points (first and last cell of the large batch), and FP64 against each
    other on the full grid to 1e-13 (the two forward paths round differently)."""
    say(f"case forward paths N={N} precision={prec}")
    big = [synth.sample_mixture(synth.mixture_anisotropic(7500 + i, 3), N, L) for i in range(128)]
    split = {24: 3, 32: 2}[N]                 # the default splits
    a = run(N, big, prec, E.EC_SCHED_FUSED, 0, split)
    b = run(N, big[:3], prec, E.EC_SCHED_FUSED, 0, split)
    op = oplan(N)
    rng = np.random.default_rng(75 + N)
    for out, c in ((a, 0), (a, 127), (b, 0), (b, 2)):
        assert np.all(np.isfinite(out[c]))
        idx = np.unique(np.concatenate([np.argsort(big[c].ravel())[-12:],
                                        rng.choice(N ** 3, 28, replace=False)]))
        q, qp, qm, _ = efm.collide_points(op, big[c], idx)
        err = np.abs(out[c].ravel()[idx] - q).max() / np.abs(qp).max()
        tol = bound_pts(prec, N, 3, qp, qm)
        say(f"  {'k_fwd3' if out is a else 'slab + x pass'} cell {c}: rel err {err:.3e} "
            f"(bound {tol:.2e})")
        assert err <= tol
    if prec == 0:
        for c in range(3):
            d = np.linalg.norm(a[c] - b[c]) / np.linalg.norm(b[c])
            say(f"  cell {c}: |batch of 128 - batch of 3| / |Q| = {d:.3e}")
            assert d <= 1e-13


@pytest.mark.parametrize("N,nmin", [(24, 96), (32, 64)])
def test_forward_kernel_threshold(N, nmin):
    """Batches of nmin - 1 and nmin cells fall on either side of the switch
    between the two-kernel forward transform and k_fwd3: their common cells
    agree on the full grid to 1e-13 (FP64, fused, default split)."""
    say(f"case forward threshold N={N}: {nmin - 1} and {nmin} cells")
    cells = [synth.sample_mixture(synth.mixture_anisotropic(7600 + i, 3), N, L) for i in range(nmin)]
    split = {24: 3, 32: 2}[N]
    a = run(N, cells[:nmin - 1], 0, E.EC_SCHED_FUSED, 0, split)
    b = run(N, cells, 0, E.EC_SCHED_FUSED, 0, split)
    for c in (0, nmin // 2, nmin - 2):
        d = np.linalg.norm(a[c] - b[c]) / np.linalg.norm(b[c])
        say(f"  cell {c}: |{nmin - 1} cells - {nmin} cells| / |Q| = {d:.3e}")
        assert np.all(np.isfinite(b[c])) and d <= 1e-13
    assert np.all(np.isfinite(b[nmin - 1]))

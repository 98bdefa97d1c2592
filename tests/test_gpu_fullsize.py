"""Parity at the headline size in the launch configuration the bench times:
1024 cells of 32^3 (hard spheres, M = 32, L = 8, R = 6, the bench's
anisotropic mixtures, seed 2001 + cell) with the schedule read from the
measured tune cache (fused passes of 1024 cells in FP64 and 512 in FP32, x
split 2), checked against the oracle: the full grid of 8 cells at pass and
workgroup-round boundaries against the plain double sum of eq. Qsk, and
sampled points of more cells against the point form.
Degenerate cells inside a fused batch: F = 0 gives Q = 0 exactly, a spike
stays finite, a Maxwellian matches the oracle.

Bars (paper_1704_07369_amd.bounds, stated a priori): FP64 1e-12 and FP32
e1 (2 + ||Q-|| / ||Q+||) of ||Q+||_2 on the full grid; on sampled points the
same numbers relative to max |Q+| over the samples (which include the points
where F peaks)."""
import os

import numpy as np
import pytest

import synth
from oracle import efm
from paper_1704_07369_amd import bounds
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
N, D, L, M, R = 32, 3, 8.0, 32, 6.0
CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1704_07369_amd", "tune_cache.txt")
_op = {}


def oplan():
    if "p" not in _op:
        _op["p"] = efm.make_plan(N, D, L, M, R=R)
    return _op["p"]


def bench_cells(n):
    return [synth.sample_mixture(synth.mixture_anisotropic(2001 + c, D), N, L) for c in range(n)]


# cells at the boundaries of the fused passes (FP64: one pass of 1024 cells;
# FP32: passes of 512) and of the workgroup rounds (two workgroups per cell,
# 256 CUs: 128 cells per round)
FULL_GRID_CELLS = [0, 127, 128, 255, 256, 511, 512, 1023]


def test_headline_batch_full_grid_vs_oracle():
    """8 cells of the 1024-cell headline batch, every grid point, against the
    oracle's plain double sum over modes (section 3.2.2, eq. Qsk), FP64 and
    FP32 in the bench's launch configuration."""
    import torch
    say("case headline batch 1024 x 32^3, full grid of 8 cells vs the double sum")
    cells = bench_cells(1024)
    p = E.Plan(N, D, L, M, R=R)
    outs = {}
    for prec in (0, 1):
        b = E.Batch([p], [1024], prec)
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.autotune(f, Q, CACHE)
        say(f"  precision {prec} schedule {b.get_schedule(0)}")
        b.collide(f, Q)
        torch.cuda.synchronize()
        outs[prec] = E.unpack(b, Q.cpu().numpy())
        b.close()
    for c in FULL_GRID_CELLS:
        ref = efm.collide_modes(oplan(), cells[c])
        den = np.linalg.norm(ref.Qplus)
        r = np.linalg.norm(ref.Qminus) / den
        e64 = np.linalg.norm(outs[0][c] - ref.Q) / den
        e32 = np.linalg.norm(outs[1][c] - ref.Q) / den
        b32 = bounds.fp32_bound(N, D, r)
        say(f"  cell {c}: FP64 {e64:.3e} (bound 1e-12), FP32 {e32:.3e} (bound {b32:.3e}), "
            f"||Q-||/||Q+|| {r:.3f}")
        assert e64 <= 1e-12
        assert e32 <= b32


@pytest.mark.parametrize("prec,check", [(0, [0, 255, 256, 511, 512, 1023]), (1, [0, 511, 512, 1023])])
def test_headline_size_parity(prec, check):
    import torch
    say(f"case full size 1024 x 32^3 precision={prec}")
    cells = bench_cells(1024)
    p = E.Plan(N, D, L, M, R=R)
    b = E.Batch([p], [1024], prec)
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.autotune(f, Q, CACHE)
    say(f"  schedule {b.get_schedule(0)}")
    b.collide(f, Q)
    torch.cuda.synchronize()
    out = E.unpack(b, Q.cpu().numpy())
    assert all(np.all(np.isfinite(o)) for o in out[::97])
    rng = np.random.default_rng(11)
    for c in check:
        idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-12:],
                                        rng.choice(N ** 3, 20, replace=False)]))
        q, qp, qm, _ = efm.collide_points(oplan(), cells[c], idx)
        tol = bounds.bound(prec, N, D, np.abs(qm).max() / np.abs(qp).max())
        err = np.abs(out[c].ravel()[idx] - q).max() / np.abs(qp).max()
        say(f"  cell {c}: max rel err {err:.3e}")
        assert err <= tol


@pytest.mark.parametrize("mode", ["fused", "terms"])
def test_degenerate_cells_in_fused_batch(mode):
    """A zero cell, a one-point spike and a Maxwellian among 33 cells, under
    the fused schedule and the term-parallel one (the default at 33 cells)."""
    import torch
    say(f"case degenerate cells in a batch of 33, {mode} schedule")
    cells = bench_cells(33)
    cells[3] = np.zeros((N,) * 3)
    spike = np.zeros((N,) * 3)
    spike[N // 2, N // 2, N // 2] = 1.0
    cells[17] = spike
    maxw = synth.Mixture(3, [synth.Gaussian(1.0, np.zeros(3), np.ones(3))])
    mx = synth.sample_mixture(maxw, N, L)
    cells[29] = mx
    p = E.Plan(N, D, L, M, R=R)
    b = E.Batch([p], [33])
    if mode == "terms":
        assert b.get_schedule(0)[0] == E.EC_SCHED_TERMS
    else:
        b.set_schedule(0, E.EC_SCHED_FUSED, 0, 0)
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    out = E.unpack(b, Q.cpu().numpy())
    assert np.all(out[3] == 0.0)
    assert np.all(np.isfinite(out[17]))
    op = oplan()
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.argsort(cells[0].ravel())[-12:], rng.choice(N ** 3, 20, replace=False)]))
    q, qp, _, _ = efm.collide_points(op, cells[0], idx)
    assert np.abs(out[0].ravel()[idx] - q).max() <= 1e-12 * np.abs(qp).max()
    # a Maxwellian: the GPU matches the oracle (the filter leaves a residual
    # that is not zero at this resolution, section 3.3; its decay with N is
    # pinned on the CPU)
    idx = np.argsort(mx.ravel())[-16:]
    q, qp, _, _ = efm.collide_points(op, mx, idx)
    assert np.abs(out[29].ravel()[idx] - q).max() <= 1e-12 * np.abs(qp).max()

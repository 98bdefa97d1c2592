"""The lines schedule (EC_SCHED_LINES: line FFTs in LDS along every axis, one
term at a time through device memory) on 64^3 and 128^3 grids, FP64:

- 64^3: full-grid agreement with the two-pass schedule (1e-13 of |Q|; a
  different transform order, the same operator), a ragged pass, and the
  in-place step;
- 64^3 and 128^3: sampled points against the oracle's point form (FP64 bar
  1e-12 of the gain; samples include the points where F peaks);
- (Table 3 row N = 128 runs through this schedule: tests/test_gpu_classical.py);
- 128^3 is FP64 and lines-only: other precisions and schedules are refused.
"""
import numpy as np
import pytest

import synth
from oracle import efm
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R, L = 6.0, 8.0


def run(p, cells, mode, chunk=0):
    import torch
    b = E.Batch([p], [len(cells)], E.EC_FP64)
    b.set_schedule(0, mode, chunk, 0)
    say(f"  schedule {b.get_schedule(0)}")
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    return E.unpack(b, Q.cpu().numpy())


def test_lines_64_matches_two_pass():
    say("case lines vs two-pass 64^3")
    p = E.Plan(64, 3, L, 8, R=R)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(9800 + i, 3), 64, L) for i in range(3)]
    a = run(p, cells, E.EC_SCHED_LINES, chunk=2)
    b = run(p, cells, E.EC_SCHED_TWO_PASS)
    for c in range(3):
        d = np.linalg.norm(a[c] - b[c]) / np.linalg.norm(b[c])
        say(f"  cell {c}: |lines - two-pass| / |Q| = {d:.3e}")
        assert np.all(np.isfinite(a[c])) and d <= 1e-13


def _sampled(op, cell, out, nrand, seed):
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([np.argsort(cell.ravel())[-12:],
                                    rng.choice(cell.size, nrand, replace=False)]))
    q, qp, _, _ = efm.collide_points(op, cell, idx)
    return np.abs(out.ravel()[idx] - q).max() / np.abs(qp).max()


@pytest.mark.parametrize("N,M,radial,ncell", [(64, 4, True, 2), (128, 1, False, 1)])
def test_lines_sampled_against_oracle(N, M, radial, ncell):
    """The oracle's tables cost O(n M') quadrature per plan: at 128^3 a
    hard-sphere plan with one direction keeps them to seconds."""
    say(f"case lines sampled vs oracle N={N} M={M} radial={radial}")
    if radial:
        p = E.Plan(N, 3, L, M, kind=E.EC_KERNEL_MAXWELL, R=R, n_radial=2, truncation="ball")
        op = efm.make_plan(N, 3, L, M, kind=efm.KIND_MAXWELL, R=R, n_radial=2, truncation="ball")
    else:
        p = E.Plan(N, 3, L, M, R=R)
        op = efm.make_plan(N, 3, L, M, R=R)
    cells = [synth.sample_mixture(synth.mixture_two_gaussians(9900 + i, 3), N, L) for i in range(ncell)]
    out = run(p, cells, E.EC_SCHED_LINES)
    for c in range(ncell):
        err = _sampled(op, cells[c], out[c], 16, N + c)
        say(f"  cell {c}: max rel err {err:.3e}")
        assert err <= 1e-12


def test_lines_step_in_place_64():
    import torch
    say("case lines step in place 64^3")
    p = E.Plan(64, 3, L, 4, R=R)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(9950 + i, 3), 64, L) for i in range(2)]
    outs = []
    for mode in (E.EC_SCHED_LINES, E.EC_SCHED_TWO_PASS):
        b = E.Batch([p], [2])
        b.set_schedule(0, mode, 0, 0)
        f = to_dev(E.pack(b, cells))
        b.step(f, 0.01, 2, None)
        torch.cuda.synchronize()
        outs.append(f.cpu().numpy())
    assert np.abs(outs[0] - outs[1]).max() <= 1e-13 * np.abs(outs[1]).max()


def test_128_is_fp64_lines_only():
    p = E.Plan(128, 3, L, 2, R=R)
    with pytest.raises(E.EcError) as ei:
        E.Batch([p], [1], E.EC_FP32)
    assert ei.value.code == E.EC_ERR_UNSUPPORTED
    b = E.Batch([p], [1], E.EC_FP64)
    assert b.get_schedule(0)[0] == E.EC_SCHED_LINES
    with pytest.raises(E.EcError) as ei:
        b.set_schedule(0, E.EC_SCHED_TWO_PASS, 0, 0)
    assert ei.value.code == E.EC_ERR_UNSUPPORTED
    p32 = E.Plan(32, 3, L, 4, R=R)
    b32 = E.Batch([p32], [1], E.EC_FP64)
    with pytest.raises(E.EcError) as ei:
        b32.set_schedule(0, E.EC_SCHED_LINES, 0, 0)
    assert ei.value.code == E.EC_ERR_UNSUPPORTED

"""Error paths of the boundary on the device: a schedule whose workspace
cannot be allocated is refused with EC_ERR_OOM and leaves the batch on its
previous schedule and workspace, which still computes the right Q."""
import numpy as np
import pytest

import synth
from oracle import efm
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R, L = 6.0, 8.0


def test_oversized_schedule_keeps_previous_workspace():
    import torch
    # 256 cells of the 64^3 sweep plan (513 transforms per evaluation): a
    # two-pass pass over all of them would need 256 x 513 x 4 MiB = 550 GB of
    # FP64 intermediates, more than the device holds
    N, M, nr, gam, ncell = 64, 64, 8, 0.5, 256
    say(f"case oversized two-pass pass: {ncell} cells of 64^3, {M}x{nr} products")
    p = E.Plan(N, 3, L, M, kind=E.EC_KERNEL_VHS, R=R, gamma=gam, n_radial=nr)
    b = E.Batch([p], [ncell], E.EC_FP64)
    b.set_schedule(0, E.EC_SCHED_TWO_PASS, 8, 0)
    before = b.get_schedule(0)
    assert before[1] == 8
    with pytest.raises(E.EcError) as ei:
        b.set_schedule(0, E.EC_SCHED_TWO_PASS, ncell, 0)
    assert ei.value.code == E.EC_ERR_OOM
    say(f"  refused: {ei.value}")
    assert b.get_schedule(0) == before
    # the batch still works on the old schedule: cell 0 a trigonometric
    # polynomial checked on the full grid, the rest zero (Q = 0)
    F0, modes = synth.trig_polynomial(7101, N, 3, L)
    cells = [F0] + [np.zeros((N,) * 3)] * (ncell - 1)
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    out = E.unpack(b, Q.cpu().numpy())
    assert np.all(out[ncell - 1] == 0.0)
    op = efm.make_plan(N, 3, L, M, kind=efm.KIND_VHS, R=R, gamma=gam, n_radial=nr, modes=modes)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([np.argsort(F0.ravel())[-16:], rng.choice(N ** 3, 48, replace=False)]))
    q, qp, _, _ = efm.collide_points(op, F0, idx)
    err = np.abs(out[0].ravel()[idx] - q).max() / np.abs(qp).max()
    say(f"  cell 0 after the refusal: max rel err {err:.3e}")
    assert err <= 1e-12
    b.close()

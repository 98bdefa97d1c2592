"""The unfiltered variant (sigma = 1, the Fourier collocation method of the
paper's positivity study, section 4.2 and Fig. 2) on the GPU: parity with
the oracle's unfiltered operator, and the contrast the figure shows -- on the
2D BKW problem the unfiltered method produces negative values (positivity
error epsilon > 0) while the entropic method keeps F >= 0 (epsilon at
roundoff)."""
import numpy as np
import pytest

import synth
from oracle import efm
from tests.gpu_util import rel_err, run_collide, say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R = 6.0
T_PAPER = efm.default_box(R)


@pytest.mark.parametrize("N,d,M", [(16, 2, 8), (16, 3, 32)])
def test_unfiltered_parity(N, d, M):
    say(f"case unfiltered parity N={N} d={d}")
    L = 8.0
    p = E.Plan(N, d, L, M, R=R, filtered=False)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(9700 + i, d), N, L) for i in range(2)]
    out, _ = run_collide(E, [p], [2], cells, E.EC_FP64)
    op = efm.make_plan(N, d, L, M, R=R, filtered=False)
    for c in range(2):
        ref = efm.collide_modes(op, cells[c])
        err = rel_err(out[c], ref.Q, ref.Qplus)
        say(f"  cell {c}: rel err {err:.3e}")
        assert err <= 1e-12


def _positivity_history(N, filtered, n_steps=100):
    import torch
    p = E.Plan(N, 2, T_PAPER, 16, R=R, filtered=filtered)
    b = E.Batch([p], [1])
    f = to_dev(E.pack(b, [synth.bkw(2, 0.0, N, T_PAPER)]))
    n = N * N
    eps = []
    for _ in range(n_steps):
        b.step(f, 0.01, 1, method="ssprk3")
        g = f[:n]
        s_abs = float(g.abs().sum())
        eps.append((s_abs - float(g.sum())) / s_abs)
    torch.cuda.synchronize()
    return np.array(eps)


@pytest.mark.parametrize("N", [16, 32])
def test_positivity_error_filtered_vs_unfiltered(N):
    say(f"case positivity study N={N}")
    e_efm = _positivity_history(N, True)
    e_fcm = _positivity_history(N, False)
    say(f"  max positivity error over t in (0, 1]: EFM {e_efm.max():.2e}, unfiltered {e_fcm.max():.2e}")
    assert e_efm.max() <= 1e-14
    assert e_fcm.max() > 1e-8

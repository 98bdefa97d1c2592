"""ec_collide_noalloc (the entry point that allocates no device memory:
its scratch is a fixed array in the library's code object) against
ec_collide on the same cells, through the C ABI: two calls in a row, the
second on fewer cells, FP64 and FP32, plus one cell against the oracle."""
import numpy as np
import pytest

import synth
from oracle import efm
from paper_1704_07369_amd import bounds
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
N, D, L, M, R = 32, 3, 8.0, 32, 6.0


def _cells(n, seed0):
    return [synth.sample_mixture(synth.mixture_anisotropic(seed0 + c, D), N, L) for c in range(n)]


def _reference(p, cells, prec):
    import torch
    b = E.Batch([p], [len(cells)], prec)
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    out = E.unpack(b, Q.cpu().numpy())
    b.close()
    return np.stack(out)


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_collide(prec):
    import torch
    say(f"case ec_collide_noalloc precision={prec}: 300 cells, then 40 cells")
    p = E.Plan(N, D, L, M, R=R)
    n = N ** D
    # first call: more cells than one pass of the scratch holds (255 in FP64)
    for ncell, seed0 in ((300, 2001), (40, 8001)):
        cells = _cells(ncell, seed0)
        ref = _reference(p, cells, prec)
        f = to_dev(np.stack(cells).ravel())
        Q = torch.full_like(f, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        E.ec_collide_noalloc(p.handle, prec, ncell, f, Q)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        out = Q.cpu().numpy().reshape(ncell, n)
        assert np.all(np.isfinite(out))
        d = np.linalg.norm(out - ref.reshape(ncell, n), axis=1) / np.linalg.norm(ref.reshape(ncell, n), axis=1)
        tol = 1e-12 if prec == 0 else bounds.fp32_bound(N, D, 3.0)
        say(f"  {ncell} cells: max rel diff vs ec_collide {d.max():.3e} (bar {tol:.1e}), "
            f"free device memory {free0} -> {free1}")
        assert d.max() <= tol
        if ncell == 40:
            assert free1 == free0        # nothing allocated on a later call
        # one cell against the oracle's point form
        op = efm.make_plan(N, D, L, M, R=R)
        c = ncell - 1
        rng = np.random.default_rng(c)
        idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-12:],
                                        rng.choice(n, 20, replace=False)]))
        q, qp, qm, _ = efm.collide_points(op, cells[c], idx)
        err = np.abs(out[c][idx] - q).max() / np.abs(qp).max()
        bar = bounds.bound(prec, N, D, np.abs(qm).max() / np.abs(qp).max())
        say(f"  cell {c} vs oracle: {err:.3e} (bound {bar:.1e})")
        assert err <= bar


def test_noalloc_rejects_what_it_cannot_run():
    import torch
    say("case ec_collide_noalloc argument checks")
    p64 = E.Plan(64, D, L, 4, R=R)          # 64^3: no fused schedule
    f = torch.zeros(2 * 64 ** 3, dtype=torch.float64, device="cuda:0")
    Q = torch.zeros_like(f)
    with pytest.raises(E.EcError) as ei:
        E.ec_collide_noalloc(p64.handle, 0, 2, f, Q)
    assert ei.value.code == E.EC_ERR_UNSUPPORTED
    p = E.Plan(N, D, L, M, R=R)
    with pytest.raises(E.EcError) as ei:
        E.ec_collide_noalloc(p.handle, 2, 1, f, Q)      # split-BF16 has no fused schedule
    assert ei.value.code == E.EC_ERR_ARG
    with pytest.raises(E.EcError) as ei:
        E.ec_collide_noalloc(p.handle, 0, 1, f, f)
    assert ei.value.code == E.EC_ERR_ARG
    E.ec_collide_noalloc(p.handle, 0, 0, f, Q)         # no cells: nothing to do

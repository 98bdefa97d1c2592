"""GPU tests of the learned surrogate: the library's FP32 forward against the
FP64 reference network, its hand-written backward against central
differences of the reference, screening with fallback to the exact operator,
and that training on the operator's own trajectories lowers the loss.

Bounds: forward 1e-5 relative (FP32 transforms of O(1) activations);
gradients 2e-3 of the largest checked component (FP32 backward against FP64
central differences)."""
import numpy as np
import pytest

import synth
from oracle import efm, fno
from tests.gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
from paper_1704_07369_amd.surrogate import Surrogate, generate_pairs, train  # noqa: E402


def _perturbed_params(sur, seed, scale=0.3):
    """Library initialisation plus seeded noise, so no block is degenerate."""
    rng = np.random.default_rng(seed)
    p = sur.params().astype(np.float64)
    N, K, C, L = sur.N, sur.modes, sur.channels, sur.layers
    for name, o, size in fno.param_blocks(N, K, C, L):
        amp = np.abs(p[o:o + size]).max() if np.any(p[o:o + size]) else 0.1
        p[o:o + size] += scale * amp * rng.standard_normal(size)
    return p.astype(np.float32)


def _inputs(N, B, seed):
    rng = np.random.default_rng(seed)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(int(rng.integers(1 << 30)), 3), N, 8.0)
             for _ in range(B)]
    h3 = (16.0 / N) ** 3
    x = np.stack([c.ravel() / (c.sum() * h3) for c in cells]).astype(np.float32)
    t = (0.01 * rng.standard_normal((B, N ** 3))).astype(np.float32)
    return x, t


@pytest.mark.parametrize("N,K,C,L,B,nfd", [(8, 2, 4, 2, 3, 48), (32, 12, 16, 4, 2, 14)])
def test_forward_and_gradients_match_reference(N, K, C, L, B, nfd):
    import torch
    say(f"case surrogate N={N} K={K} C={C} L={L}")
    sur = Surrogate(N, K, C, L, seed=7, max_batch=B)
    p = _perturbed_params(sur, 11)
    sur.set_params(p)
    x, t = _inputs(N, B, 5)
    xd, td = to_dev(x), to_dev(t)
    y = torch.zeros_like(xd)
    sur.forward(xd, y, B)
    torch.cuda.synchronize()
    yref = fno.forward(p.astype(np.float64), x.astype(np.float64), N, K, C, L)
    err = np.abs(y.cpu().numpy() - yref).max() / np.abs(yref).max()
    say(f"  forward rel err {err:.3e}")
    assert err < 1e-5
    loss = sur.train_step(xd, td, B, 0.0, update=False, want_loss=True)
    lref = fno.loss(p.astype(np.float64), x, t, N, K, C, L)
    say(f"  loss {loss:.6e} ref {lref:.6e}")
    assert abs(loss - lref) < 1e-5 * abs(lref)
    g = sur.grads().astype(np.float64)
    rng = np.random.default_rng(3)
    idx = []
    for name, o, size in fno.param_blocks(N, K, C, L):
        k = max(1, nfd // len(fno.param_blocks(N, K, C, L)))
        idx += list(o + rng.choice(size, min(k, size), replace=False))
    # for the spectral blocks also check the largest gradient entries
    for name, o, size in fno.param_blocks(N, K, C, L):
        if name.startswith("R"):
            idx += list(o + np.argsort(-np.abs(g[o:o + size]))[:2])
    gfd = fno.fd_grad(p.astype(np.float64), x, t, N, K, C, L, idx)
    scale = np.abs(gfd).max()
    err = np.abs(g[idx] - gfd).max() / scale
    say(f"  gradient check on {len(idx)} parameters: max err {err:.3e} (scale {scale:.3e})")
    assert err < 2e-3


def test_forward_over_several_mixing_chunks():
    """The mode mixing at 16 channels runs on the matrix cores with one wave
    per mode and 64 cells: a batch of 67 cells (one full chunk and a ragged
    one of 3) at the production size (32^3, 12 modes, 16 channels, one layer)
    against the FP64 reference network, every cell within the forward bound."""
    import torch
    N, K, C, L, B = 32, 12, 16, 1, 67
    say(f"case surrogate forward N={N} K={K} C={C} L={L} B={B}")
    sur = Surrogate(N, K, C, L, seed=9, max_batch=B)
    p = _perturbed_params(sur, 13)
    sur.set_params(p)
    x, _ = _inputs(N, B, 8)
    xd = to_dev(x)
    y = torch.zeros_like(xd)
    sur.forward(xd, y, B)
    torch.cuda.synchronize()
    yref = fno.forward(p.astype(np.float64), x.astype(np.float64), N, K, C, L)
    err = np.abs(y.cpu().numpy() - yref).max(axis=1) / np.abs(yref).max(axis=1)
    say(f"  per-cell forward rel err: max {err.max():.3e} (cells 0, 63, 64, 66: "
        f"{err[0]:.2e} {err[63]:.2e} {err[64]:.2e} {err[66]:.2e})")
    assert err.max() < 1e-5


def test_screen_fallback_matches_exact_operator():
    """A corrupted network (NaN weights) fails the screen on every cell, and
    the fallback returns the exact operator's Q."""
    import torch
    say("case screen fallback")
    N, L, M = 16, 8.0, 32
    plan = E.Plan(N, 3, L, M, R=6.0)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(500 + i, 3), N, L) for i in range(5)]
    b = E.Batch([plan], [5])
    f = to_dev(E.pack(b, cells))
    Qe = torch.zeros_like(f)
    b.collide(f, Qe)
    sur = Surrogate(N, 6, 8, 2, seed=3, max_batch=2)
    bad = sur.params()
    bad[:] = np.nan
    sur.set_params(bad)
    Qs = torch.zeros_like(f)
    fell = torch.zeros(5, dtype=torch.int32, device="cuda")
    scr = torch.zeros(5 * 4, dtype=torch.float64, device="cuda")
    nf = sur.collide(b, f, Qs, fell_back=fell, screen=scr)
    torch.cuda.synchronize()
    assert nf == 5 and fell.cpu().numpy().tolist() == [1] * 5
    qe, qs = E.unpack(b, Qe.cpu().numpy()), E.unpack(b, Qs.cpu().numpy())
    for c in range(5):
        assert np.abs(qs[c] - qe[c]).max() <= 1e-14 * np.abs(qe[c]).max()
    # the exact operator itself passes the screen (its own H-functional <= 0,
    # mass residual ~1e-16; momentum/energy defects are small)
    op = efm.make_plan(N, 3, L, M, R=6.0)
    for c in range(5):
        m = efm.monitors(op, cells[c], qe[c])
        assert m["entropy_prod"] <= 0 and abs(m["sumQ"]) <= 1e-3 * m["sumabsQ"]


def test_training_on_operator_trajectories_lowers_loss():
    import torch
    say("case surrogate training (16^3)")
    N, L, M = 16, 8.0, 32
    plan = E.Plan(N, 3, L, M, R=6.0)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(5001 + i, 3), N, L) for i in range(16)]
    sur = Surrogate(N, 6, 8, 4, seed=1, max_batch=8)
    Fin, Tgt = generate_pairs(torch, plan, cells, 8, 0.01, sur)
    assert Fin.shape == (128, N ** 3) and torch.isfinite(Tgt).all()
    l0 = sur.train_step(Fin[:8], Tgt[:8], 8, 0.0, update=False, want_loss=True)
    p0 = sur.params()
    hist, steps = train(torch, sur, Fin, Tgt, seconds=8.0, batch=8, lr=2e-3)
    l1 = sur.train_step(Fin[:8], Tgt[:8], 8, 0.0, update=False, want_loss=True)
    say(f"  steps {steps}: loss {l0:.3e} -> {l1:.3e}")
    assert l1 < 0.5 * l0
    # held-out cells (fresh seeds): projected prediction against the exact
    # operator, trained network against its own initialisation
    test = [synth.sample_mixture(synth.mixture_anisotropic(6001 + i, 3), N, L) for i in range(8)]
    b = E.Batch([plan], [8])
    f = to_dev(E.pack(b, test))
    Qe = torch.zeros_like(f)
    b.collide(f, Qe)
    Qs = torch.zeros_like(f)

    def held_out_error():
        sur.collide(b, f, Qs, tau_m=-1.0)
        torch.cuda.synchronize()
        d = (Qs - Qe).view(8, -1).norm(dim=1) / Qe.view(8, -1).norm(dim=1)
        return float(d.median())

    e1 = held_out_error()
    trained = sur.params()
    sur.set_params(p0)
    e0 = held_out_error()
    sur.set_params(trained)
    say(f"  held-out median rel L2 error: initial {e0:.3e}, trained {e1:.3e}")
    assert e1 < 0.3 and e1 < 0.2 * e0


def test_mass_projection_matches_reference():
    """Screen disabled: the library's Q is the FP64 mass projection of its own
    network output (reference: oracle/fno.py on the same FP32 prediction),
    its mass vanishes, and the residuals it reports are those of the
    unprojected prediction."""
    import torch
    say("case surrogate projection")
    N, L, M = 16, 8.0, 32
    plan = E.Plan(N, 3, L, M, R=6.0)
    nc = 5
    cells = [synth.sample_mixture(synth.mixture_anisotropic(700 + i, 3), N, L) for i in range(nc)]
    b = E.Batch([plan], [nc])
    f = to_dev(E.pack(b, cells))
    sur = Surrogate(N, 6, 8, 2, seed=5, max_batch=2)
    xin = torch.empty((nc, N ** 3), dtype=torch.float32, device="cuda")
    y = torch.empty_like(xin)
    for c in range(0, nc, 2):
        k = min(2, nc - c)
        sur.prepare(b, f, None, c, k, xin[c:c + k], None)
        sur.forward(xin[c:c + k], y[c:c + k], k)
    Qs = torch.zeros_like(f)
    fell = torch.ones(nc, dtype=torch.int32, device="cuda")
    scr = torch.zeros(nc * 4, dtype=torch.float64, device="cuda")
    nf = sur.collide(b, f, Qs, tau_m=-1.0, fell_back=fell, screen=scr)
    torch.cuda.synchronize()
    assert nf == 0 and fell.cpu().numpy().tolist() == [0] * nc
    h3 = (2 * L / N) ** 3
    c0 = (2 * np.pi) ** 1.5
    yh = y.cpu().numpy().astype(np.float64)
    qs = E.unpack(b, Qs.cpu().numpy())
    v = -L + np.arange(N) * (2 * L / N)
    vx, vy, vz = np.meshgrid(v, v, v, indexing="ij")
    for c in range(nc):
        mass = h3 * cells[c].sum()
        raw = (yh[c] * mass ** 2 / c0 ** 2).reshape(N, N, N)
        ref = fno.mass_projection(raw)
        err = np.abs(qs[c] - ref).max() / np.abs(ref).max()
        say(f"  cell {c}: projection rel err {err:.2e}")
        assert err < 1e-10
        q = qs[c]
        assert abs(q.sum()) < 1e-12 * np.abs(q).sum()
        ra = np.abs(raw).sum()
        res = [abs(raw.sum()) / ra,
               np.sqrt((raw * vx).sum() ** 2 + (raw * vy).sum() ** 2 + (raw * vz).sum() ** 2) / (L * ra),
               abs((raw * (vx**2 + vy**2 + vz**2)).sum()) / (3 * L * L * ra)]
        got = scr.cpu().numpy()[c * 4 + 1:c * 4 + 4]
        assert np.allclose(got, res, rtol=1e-8, atol=1e-14), (got, res)


def test_screen_flags_follow_the_stated_rule():
    """ec_surrogate_collide's screen: a cell falls back unless the projected
    Q's H-functional is <= 0, the raw mass residual <= tau_m and, when
    tau_e >= 0, the momentum and energy residuals <= tau_e.  Checked flag by
    flag against the screen values it reports, for tau_e < 0 (the default:
    no moment checks) and for a tau_e that every cell fails; fallen-back
    cells carry the exact operator's Q."""
    import torch
    from paper_1704_07369_amd.surrogate import SCREEN_TAU_E, SCREEN_TAU_M
    say("case surrogate screen rule")
    N, L, M = 16, 8.0, 32
    plan = E.Plan(N, 3, L, M, R=6.0)
    nc = 6
    cells = [synth.sample_mixture(synth.mixture_anisotropic(900 + i, 3), N, L) for i in range(nc)]
    b = E.Batch([plan], [nc])
    f = to_dev(E.pack(b, cells))
    Qe = torch.zeros_like(f)
    b.collide(f, Qe)
    sur = Surrogate(N, 6, 8, 2, seed=3, max_batch=4)
    qe = E.unpack(b, Qe.cpu().numpy())
    assert SCREEN_TAU_E < 0 and SCREEN_TAU_M > 0
    for tau_m, tau_e in ((SCREEN_TAU_M, SCREEN_TAU_E), (1.0, 1e-12), (1.0, -1.0)):
        Qs = torch.zeros_like(f)
        fell = torch.zeros(nc, dtype=torch.int32, device="cuda")
        scr = torch.zeros(nc * 4, dtype=torch.float64, device="cuda")
        nf = sur.collide(b, f, Qs, tau_m=tau_m, tau_e=tau_e, fell_back=fell, screen=scr)
        torch.cuda.synchronize()
        s = scr.cpu().numpy().reshape(nc, 4)
        ok = (s[:, 0] <= 0) & (s[:, 1] <= tau_m)
        if tau_e >= 0:
            ok &= (s[:, 2] <= tau_e) & (s[:, 3] <= tau_e)
        fl = fell.cpu().numpy()
        say(f"  tau_m {tau_m} tau_e {tau_e}: fallback {fl.tolist()}")
        assert fl.tolist() == (~ok).astype(int).tolist() and nf == int((~ok).sum())
        if tau_e == 1e-12:
            assert nf == nc
        qs = E.unpack(b, Qs.cpu().numpy())
        for c in np.nonzero(fl)[0]:
            assert np.abs(qs[c] - qe[c]).max() <= 1e-14 * np.abs(qe[c]).max()

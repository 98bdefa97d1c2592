"""GPU parity of the HIP collision operator against the CPU oracle.

Bar (FP64): ||Q_gpu - Q_oracle||_2 / ||Q+_oracle||_2 <= 1e-12 per cell (full
grid), or max_r |Q_gpu - Q_oracle| / max_r |Q+_oracle| <= 1e-12 over sampled
points at large sizes.  The normaliser is the gain because Q itself nearly
vanishes near equilibrium while the rounding of the transforms scales with
the gain.  FP32 transforms and the split-BF16 x pass: the per-size bounds
stated a priori in paper_1704_07369_amd.bounds (worst-case rounding growth
over the forward and inverse stages, doubled by the product a_t b_t, plus the
loss term's share).
"""
import math

import numpy as np
import pytest

import synth
from oracle import efm
from tests.gpu_util import bound_full, bound_pts, rel_err, run_collide, say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R = 6.0
TOL64 = 1e-12

_oracle_plans = {}


def oplan(N, d, L, M):
    key = (N, d, L, M)
    if key not in _oracle_plans:
        _oracle_plans[key] = efm.make_plan(N, d, L, M, R=R)
    return _oracle_plans[key]


def mixtures(d, N, L, n, seed0):
    return [synth.sample_mixture(synth.mixture_anisotropic(seed0 + i, d), N, L) for i in range(n)]


@pytest.mark.parametrize("N,d,M,L,ncell", [
    (8, 3, 8, 8.0, 3), (12, 3, 32, 8.0, 2), (16, 3, 32, 8.0, 3),
    (8, 2, 3, efm.default_box(R), 2), (16, 2, 4, 8.0, 3), (32, 2, 16, 8.0, 2), (24, 2, 5, 8.0, 1),
])
def test_fp64_full_grid_parity(N, d, M, L, ncell):
    say(f"case fp64 full grid N={N} d={d} M={M} cells={ncell}")
    p = E.Plan(N, d, L, M, R=R)
    cells = mixtures(d, N, L, ncell, 1000 + N)
    out, _ = run_collide(E, [p], [ncell], cells, E.EC_FP64)
    op = oplan(N, d, L, M)
    for c in range(ncell):
        ref = efm.collide_modes(op, cells[c])
        err = rel_err(out[c], ref.Q, ref.Qplus)
        say(f"  cell {c}: rel err {err:.3e}")
        assert err <= TOL64


@pytest.mark.parametrize("N,M,ncell,chunk", [(24, 32, 3, 2), (32, 32, 3, 2)])
def test_fp64_sampled_parity_large(N, M, ncell, chunk):
    """24^3 and 32^3 with a pass size that leaves a ragged last pass."""
    say(f"case fp64 sampled N={N} M={M} cells={ncell} chunk={chunk}")
    L = 8.0
    p = E.Plan(N, 3, L, M, R=R)
    cells = mixtures(3, N, L, ncell, 2000 + N)
    out, _ = run_collide(E, [p], [ncell], cells, E.EC_FP64, chunks={0: chunk})
    op = oplan(N, 3, L, M)
    rng = np.random.default_rng(N)
    for c in range(ncell):
        idx = rng.choice(N ** 3, 48, replace=False)
        q, qp, _, _ = efm.collide_points(op, cells[c], idx)
        err = np.abs(out[c].ravel()[idx] - q).max() / np.abs(qp).max()
        say(f"  cell {c}: max rel err {err:.3e}")
        assert err <= TOL64


@pytest.mark.parametrize("mode,chunk,G", [(0, 1, 1), (0, 2, 3), (0, 3, 33), (0, 0, 0), (1, 2, 0)])
def test_schedules_parity(mode, chunk, G):
    """Pipelined schedule (ragged chunks, term groups from 1 to J) and the
    two-pass schedule give the same operator (5 cells of 16^3)."""
    say(f"case schedule mode={mode} chunk={chunk} G={G}")
    import torch
    L, N, M, ncell = 8.0, 16, 32, 5
    p = E.Plan(N, 3, L, M, R=R)
    cells = mixtures(3, N, L, ncell, 7000)
    b = E.Batch([p], [ncell])
    b.set_schedule(0, mode, chunk, G)
    say(f"  schedule {b.get_schedule(0)}")
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    out = E.unpack(b, Q.cpu().numpy())
    op = oplan(N, 3, L, M)
    for c in range(ncell):
        ref = efm.collide_modes(op, cells[c])
        err = rel_err(out[c], ref.Q, ref.Qplus)
        say(f"  cell {c}: rel err {err:.3e}")
        assert err <= TOL64


def test_fp32_parity():
    say("case fp32 16^3 and 2D 32^2")
    for (N, d, M, L) in [(16, 3, 32, 8.0), (32, 2, 16, 8.0)]:
        p = E.Plan(N, d, L, M, R=R)
        cells = mixtures(d, N, L, 2, 3000 + N)
        out, _ = run_collide(E, [p], [2], cells, E.EC_FP32)
        op = oplan(N, d, L, M)
        for c in range(2):
            ref = efm.collide_modes(op, cells[c])
            err = rel_err(out[c], ref.Q, ref.Qplus)
            tol = bound_full(1, N, d, ref)
            say(f"  N={N} d={d} cell {c}: rel err {err:.3e} (bound {tol:.2e})")
            assert err <= tol


def test_bf16x3_parity():
    """Split-BF16 MFMA x pass: 16^3 full grid and 32^3 sampled points."""
    say("case bf16x3")
    for (N, ncell) in [(16, 2), (32, 2)]:
        L = 8.0
        p = E.Plan(N, 3, L, 32, R=R)
        cells = mixtures(3, N, L, ncell, 9000 + N)
        out, _ = run_collide(E, [p], [ncell], cells, E.EC_BF16X3)
        op = oplan(N, 3, L, 32)
        for c in range(ncell):
            if N == 16:
                ref = efm.collide_modes(op, cells[c])
                err = rel_err(out[c], ref.Q, ref.Qplus)
                tol = bound_full(2, N, 3, ref)
            else:
                idx = np.random.default_rng(c).choice(N ** 3, 48, replace=False)
                q, qp, qm, _ = efm.collide_points(op, cells[c], idx)
                err = np.abs(out[c].ravel()[idx] - q).max() / np.abs(qp).max()
                tol = bound_pts(2, N, 3, qp, qm)
            say(f"  N={N} cell {c}: rel err {err:.3e} (bound {tol:.2e})")
            assert err <= tol


def test_bf16x3_rejects_unsupported_sizes():
    say("case bf16x3 unsupported")
    for (N, d) in [(24, 3), (16, 2)]:
        p = E.Plan(N, d, 8.0, 8, R=R)
        with pytest.raises(E.EcError) as ei:
            E.Batch([p], [1], E.EC_BF16X3)
        assert ei.value.code == E.EC_ERR_UNSUPPORTED


def test_mixed_batch_parity():
    """Groups of 16^3, 24^3 and 32^3 cells in one batch (and an empty group)."""
    say("case mixed batch 16/24/32 + empty group")
    L = 8.0
    plans = [E.Plan(16, 3, L, 32, R=R), E.Plan(8, 3, L, 8, R=R), E.Plan(24, 3, L, 32, R=R),
             E.Plan(32, 3, L, 32, R=R)]
    counts = [2, 0, 2, 1]
    sizes = [16, 16, 24, 24, 32]
    cells = [synth.sample_mixture(synth.mixture_anisotropic(4000 + i, 3), N, L) for i, N in enumerate(sizes)]
    out, _ = run_collide(E, plans, counts, cells, E.EC_FP64)
    rng = np.random.default_rng(1)
    for c, N in enumerate(sizes):
        idx = rng.choice(N ** 3, 32, replace=False)
        q, qp, _, _ = efm.collide_points(oplan(N, 3, L, 32), cells[c], idx)
        err = np.abs(out[c].ravel()[idx] - q).max() / np.abs(qp).max()
        say(f"  cell {c} N={N}: max rel err {err:.3e}")
        assert err <= TOL64


def test_edge_inputs():
    """F = 0 gives Q = 0; F with a vanishing region keeps Q >= 0 there
    (proof of Theorem 1); a delta-like cell stays finite."""
    say("case edge inputs")
    import torch
    N, L, M = 16, 8.0, 8
    p = E.Plan(N, 2, L, M, R=R)
    zero = np.zeros((N, N))
    holey = synth.sample_mixture(synth.mixture_two_gaussians(5, 2), N, L)
    holey[2:7, 3:11] = 0.0
    spike = np.zeros((N, N)); spike[N // 2, N // 2] = 1.0
    out, _ = run_collide(E, [p], [3], [zero, holey, spike], E.EC_FP64)
    assert np.all(out[0] == 0.0)
    ref = efm.collide_modes(oplan(N, 2, L, M), holey)
    assert rel_err(out[1], ref.Q, ref.Qplus) <= TOL64
    z = holey == 0.0
    assert out[1][z].min() >= -1e-13 * np.abs(ref.Qplus).max()
    assert np.all(np.isfinite(out[2]))


def test_alias_rejected():
    say("case alias rejected")
    import torch
    p = E.Plan(8, 3, 8.0, 8, R=R)
    b = E.Batch([p], [1])
    f = torch.zeros(b.n_elems, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EcError) as ei:
        b.collide(f, f)
    assert ei.value.code == E.EC_ERR_ARG


def test_monitors_and_entropy_production():
    say("case monitors")
    import torch
    N, L, M = 12, 8.0, 32
    p = E.Plan(N, 3, L, M, R=R)
    cells = mixtures(3, N, L, 3, 5000)
    cells[2][0, :, :] = 0.0
    b = E.Batch([p], [3])
    f = to_dev(E.pack(b, cells))
    Q = torch.zeros_like(f)
    b.collide(f, Q)
    mon = torch.zeros(3 * E.EC_NMON, dtype=torch.float64, device="cuda")
    ep = torch.zeros(3, dtype=torch.float64, device="cuda")
    nn = torch.zeros(3, dtype=torch.int32, device="cuda")
    b.monitors(f, Q, mon)
    b.entropy_prod(f, Q, ep, nn)
    torch.cuda.synchronize()
    qs = E.unpack(b, Q.cpu().numpy())
    mon = mon.cpu().numpy().reshape(3, E.EC_NMON)
    op = oplan(N, 3, L, M)
    for c in range(3):
        m = efm.monitors(op, cells[c], qs[c])
        assert mon[c, 0] == pytest.approx(m["mass"], rel=1e-13)
        assert abs(mon[c, 1] - m["sumQ"]) <= 1e-13 * m["sumabsQ"]
        assert mon[c, 2] == pytest.approx(m["entropy_prod"], rel=1e-12, abs=1e-15)
        assert mon[c, 3] == pytest.approx(m["eta"], rel=1e-13)
        assert mon[c, 4] == m["minF"]
        assert mon[c, 6] == pytest.approx(m["sumabsQ"], rel=1e-13)
        # momentum and energy of Q (reported, not conserved): sums of the same
        # terms in another order, scale h^d sum |Q| |v| and h^d sum |Q| |v|^2
        h3 = (2.0 * L / N) ** 3
        vmax = L * math.sqrt(3.0)
        for i in range(3):
            assert abs(mon[c, 7 + i] - m["momentum"][i]) <= 1e-13 * h3 * m["sumabsQ"] * vmax
        assert abs(mon[c, 10] - m["energy"]) <= 1e-13 * h3 * m["sumabsQ"] * vmax ** 2
        assert ep[c].item() == pytest.approx(m["entropy_prod"], rel=1e-12, abs=1e-15)
        assert nn[c].item() == m["n_nonpos"]
        assert ep[c].item() <= 0.0                       # discrete H-theorem
        assert abs(mon[c, 1]) <= 1e-13 * mon[c, 6]       # mass conservation


def test_step_graph_matches_oracle_euler():
    """ec_step (graph-captured forward Euler) against the oracle's FE steps."""
    say("case step graph")
    import torch
    N, L, M, dt, steps = 8, 8.0, 8, 0.01, 5
    p = E.Plan(N, 3, L, M, R=R)
    cells = mixtures(3, N, L, 2, 6000)
    b = E.Batch([p], [2])
    f = to_dev(E.pack(b, cells))
    mon = torch.zeros(steps * 2 * 2, dtype=torch.float64, device="cuda")
    b.step(f, dt, steps, mon)
    torch.cuda.synchronize()
    got = E.unpack(b, f.cpu().numpy())
    monh = mon.cpu().numpy().reshape(steps, 2, 2)
    op = oplan(N, 3, L, M)
    for c in range(2):
        F = cells[c].copy()
        for s in range(steps):
            F = efm.fe_step(lambda u: efm.collide_modes(op, u).Q, F, dt)
            m = efm.monitors(op, F, np.zeros_like(F))
            assert monh[s, c, 0] == pytest.approx(m["mass"], rel=1e-12)
            assert monh[s, c, 1] == pytest.approx(m["eta"], rel=1e-11)
        assert np.abs(got[c] - F).max() <= 1e-12 * np.abs(F).max()
    # a second call replays the cached graph from the new state
    b.step(f, dt, 1, mon)
    torch.cuda.synchronize()


@pytest.mark.parametrize("N,M,ncell,prec", [(32, 16, 1, 0), (32, 16, 5, 0), (16, 8, 3, 0),
                                            (32, 16, 3, 1), (24, 8, 2, 0)])
def test_2d_term_parallel(N, M, ncell, prec):
    """Small 2D batches default to the term-parallel schedule (one block per
    (cell, term), partial products summed in the fixed order loss-first):
    the full grid against the oracle's double sum, against the two-pass
    schedule on the same cells, and three forward-Euler steps of the captured
    graph against the two-pass schedule's."""
    import torch
    say(f"case 2D term-parallel N={N} M={M} cells={ncell} precision={prec}")
    L = 8.0
    p = E.Plan(N, 2, L, M, R=R)
    cells = mixtures(2, N, L, ncell, 4400 + N)
    if ncell > 1:
        cells[1] = synth.bkw_datum(2, N, L)
    outs, steps = {}, {}
    for mode in (E.EC_SCHED_TERMS, E.EC_SCHED_TWO_PASS):
        b = E.Batch([p], [ncell], prec)
        if mode == E.EC_SCHED_TWO_PASS:
            b.set_schedule(0, mode, 0, 0)
        say(f"  schedule {b.get_schedule(0)}")
        assert b.get_schedule(0)[0] == mode
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.collide(f, Q)
        b.step(f, 0.01, 3)
        torch.cuda.synchronize()
        outs[mode] = E.unpack(b, Q.cpu().numpy())
        steps[mode] = E.unpack(b, f.cpu().numpy())
        b.close()
    op = oplan(N, 2, L, M)
    for c in range(ncell):
        qt, q2 = outs[E.EC_SCHED_TERMS][c], outs[E.EC_SCHED_TWO_PASS][c]
        ref = efm.collide_modes(op, cells[c])
        err = rel_err(qt, ref.Q, ref.Qplus)
        tol = bound_full(prec, N, 2, ref)
        d2 = np.abs(qt - q2).max() / np.abs(ref.Qplus).max()
        ds = np.abs(steps[E.EC_SCHED_TERMS][c] - steps[E.EC_SCHED_TWO_PASS][c]).max()
        say(f"  cell {c}: vs oracle {err:.2e} (bound {tol:.1e}), vs two-pass {d2:.1e}, "
            f"3 steps vs two-pass {ds:.1e}")
        assert err <= tol
        assert d2 <= (1e-14 if prec == 0 else 1e-6)
        assert ds <= (1e-14 if prec == 0 else 1e-6) * np.abs(steps[E.EC_SCHED_TWO_PASS][c]).max()

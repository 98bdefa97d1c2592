"""The term-parallel schedule (EC_SCHED_TERMS; 32^3 column kernel, 16^3 and
24^3 LDS-volume kernel): one workgroup per (cell, term, x residue class)
writes its term's products, a second kernel sums them per point in the
fused kernel's order.

- against the fused schedule on the same inputs: the same sums of the same
  FP64 products, so agreement to 1e-14 of the gain in FP64 and FP32 (only
  the contraction of the last product into its sum may differ);
- against the CPU oracle at sampled points (the 16 largest-F points among
  them): FP64 1e-12, FP32 its stated per-size bound (bounds.py) of the
  gain's scale;
- ragged passes (chunk below the cell count), splits 2 and 4, a single cell;
- three forward-Euler steps replayed from the captured graph equal three
  steps of the fused schedule, also for a batch of small 16^3, 24^3 and
  32^3 groups that all start on this schedule."""
import numpy as np
import pytest

import synth
from oracle import efm
from tests.gpu_util import bound_pts, say, to_dev

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
N, R, L, M = 32, 6.0, 8.0, 32


def _cells(n, seed):
    return [synth.sample_mixture(synth.mixture_anisotropic(seed + i, 3), N, L) for i in range(n)]


def _run(plan, cells, prec, mode, chunk, split, steps=0):
    import torch
    b = E.Batch([plan], [len(cells)], prec)
    b.set_schedule(0, mode, chunk, split)
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    if steps:
        b.step(f, 0.01, steps, None)
    torch.cuda.synchronize()
    return E.unpack(b, Q.cpu().numpy()), E.unpack(b, f.cpu().numpy()), b.get_schedule(0)


@pytest.mark.parametrize("prec,split,chunk,ncell", [
    (0, 2, 0, 1), (0, 2, 2, 3), (0, 4, 0, 2), (1, 2, 0, 1), (1, 4, 3, 5),
])
def test_terms_match_fused_and_oracle(prec, split, chunk, ncell):
    say(f"case term-parallel 32^3 precision={prec} split={split} chunk={chunk} cells={ncell}")
    plan = E.Plan(N, 3, L, M, R=R)
    cells = _cells(ncell, 8100 + 10 * split + ncell)
    qt, ft, sched = _run(plan, cells, prec, E.EC_SCHED_TERMS, chunk, split, steps=3)
    qf, ff, _ = _run(plan, cells, prec, E.EC_SCHED_FUSED, 0, split, steps=3)
    say(f"  schedule {sched}")
    assert sched[0] == E.EC_SCHED_TERMS and sched[2] == split
    op = efm.make_plan(N, 3, L, M, R=R)
    rng = np.random.default_rng(prec + split)
    for c in range(ncell):
        assert np.all(np.isfinite(qt[c]))
        scale = np.abs(qf[c]).max()
        d_fused = np.abs(qt[c] - qf[c]).max() / scale
        d_step = np.abs(ft[c] - ff[c]).max() / np.abs(ff[c]).max()
        idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-16:],
                                        rng.choice(N ** 3, 48, replace=False)]))
        q, qp, qm, _ = efm.collide_points(op, cells[c], idx)
        err = np.abs(qt[c].ravel()[idx] - q).max() / np.abs(qp).max()
        say(f"  cell {c}: vs fused {d_fused:.2e}, 3 steps vs fused {d_step:.2e}, "
            f"vs oracle {err:.2e}")
        assert d_fused <= 1e-14 and d_step <= 1e-14
        assert err <= bound_pts(prec, N, 3, qp, qm)


def test_terms_is_the_small_batch_default_and_validated():
    say("case term-parallel default and rejections")
    plan = E.Plan(N, 3, L, M, R=R)
    b = E.Batch([plan], [4], E.EC_FP64)
    assert b.get_schedule(0)[0] == E.EC_SCHED_TERMS
    with pytest.raises(E.EcError):
        b.set_schedule(0, E.EC_SCHED_TERMS, 0, 3)
    p16 = E.Plan(16, 3, L, M, R=R)
    b16 = E.Batch([p16], [2], E.EC_FP64)
    assert b16.get_schedule(0)[0] == E.EC_SCHED_TERMS
    with pytest.raises(E.EcError):
        b16.set_schedule(0, E.EC_SCHED_TERMS, 0, 4)       # not a split of 16^3
    p64 = E.Plan(64, 3, L, 8, R=R)
    b64 = E.Batch([p64], [1], E.EC_FP64)
    with pytest.raises(E.EcError):
        b64.set_schedule(0, E.EC_SCHED_TERMS, 0, 0)
    bb = E.Batch([plan], [2], E.EC_BF16X3)
    with pytest.raises(E.EcError):
        bb.set_schedule(0, E.EC_SCHED_TERMS, 0, 0)


def test_small_batch_defaults_of_other_sizes():
    """Default schedules by group size: term-parallel up to the measured
    crossover (FP64 / FP32: 16^3 192 / 192 cells, 24^3 64 / 80, 32^3 48 / 40),
    fused above it (x split 4 for 32^3 launches of up to CUs / 4 cells, 2 for
    24^3 launches where 2 workgroups per cell fill one round and 3 do not),
    two-pass at 64^3; 2D grids of N <= 32 term-parallel up to 1024 cells (the
    2D form: one block per cell and term), two-pass above."""
    say("case small-batch defaults of other sizes")
    T, F = E.EC_SCHED_TERMS, E.EC_SCHED_FUSED
    for N, d, prec, count, want in [
            (16, 3, 0, 2, T), (24, 3, 0, 2, T), (16, 3, 0, 192, T), (16, 3, 0, 193, F),
            (16, 3, 1, 192, T), (16, 3, 1, 193, F), (24, 3, 0, 64, T), (24, 3, 0, 65, F),
            (24, 3, 1, 80, T), (24, 3, 1, 81, F), (32, 3, 0, 48, T), (32, 3, 0, 49, F),
            (32, 3, 1, 40, T), (32, 3, 1, 41, F),
            (64, 3, 0, 2, E.EC_SCHED_TWO_PASS), (32, 2, 0, 2, T), (32, 2, 1, 1024, T),
            (32, 2, 0, 1025, E.EC_SCHED_TWO_PASS)]:
        p = E.Plan(N, d, L, 8, R=R)
        b = E.Batch([p], [count], prec)
        say(f"  N={N} d={d} precision={prec} cells={count}: schedule {b.get_schedule(0)}")
        assert b.get_schedule(0)[0] == want
        b.close()
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for N, count, split in [(32, cus // 4, 4), (32, cus // 4 + 1, 2), (32, 1024, 2),
                            (24, cus // 3 + 1, 2), (24, cus // 2, 2), (24, cus // 2 + 1, 3)]:
        b = E.Batch([E.Plan(N, 3, L, 8, R=R)], [count], E.EC_FP64)
        b.set_schedule(0, E.EC_SCHED_FUSED, 0, 0)
        say(f"  fused N={N} cells={count} (CUs {cus}): schedule {b.get_schedule(0)}")
        assert b.get_schedule(0)[2] == split
        b.close()


@pytest.mark.parametrize("Nl,prec,split,ncell", [
    (16, 0, 1, 2), (16, 0, 2, 3), (16, 1, 1, 2), (24, 0, 3, 2), (24, 0, 2, 3), (24, 1, 3, 1),
])
def test_terms_lds_volume_form(Nl, prec, split, ncell):
    """N = 16, 24: the term-parallel form of the LDS-volume kernel against the
    fused schedule (same products, same order of the sums) and the oracle."""
    import torch
    say(f"case term-parallel {Nl}^3 precision={prec} split={split} cells={ncell}")
    plan = E.Plan(Nl, 3, L, M, R=R)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(8300 + Nl + i, 3), Nl, L)
             for i in range(ncell)]
    out = {}
    for mode in (E.EC_SCHED_TERMS, E.EC_SCHED_FUSED):
        b = E.Batch([plan], [ncell], prec)
        b.set_schedule(0, mode, 0, split)
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.collide(f, Q)
        torch.cuda.synchronize()
        out[mode] = E.unpack(b, Q.cpu().numpy())
    op = efm.make_plan(Nl, 3, L, M, R=R)
    rng = np.random.default_rng(Nl + split)
    for c in range(ncell):
        qt, qf = out[E.EC_SCHED_TERMS][c], out[E.EC_SCHED_FUSED][c]
        d_fused = np.abs(qt - qf).max() / np.abs(qf).max()
        idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-16:],
                                        rng.choice(Nl ** 3, 48, replace=False)]))
        q, qp, qm, _ = efm.collide_points(op, cells[c], idx)
        err = np.abs(qt.ravel()[idx] - q).max() / np.abs(qp).max()
        say(f"  cell {c}: vs fused {d_fused:.2e}, vs oracle {err:.2e}")
        assert d_fused <= 1e-14 and err <= bound_pts(prec, Nl, 3, qp, qm)


def test_mixed_small_groups_default_to_terms_and_step_like_fused():
    """A batch of small 16^3, 24^3 and 32^3 groups starts every group on the
    term-parallel schedule; one evaluation and three graph-replayed
    forward-Euler steps (a ragged pass at 16^3) equal those of the fused
    schedule at the same x splits."""
    import torch
    say("case mixed small groups 16^3 x 3, 24^3 x 2, 32^3 x 2, term-parallel vs fused")
    sizes, counts = [16, 24, 32], [3, 2, 2]
    plans = [E.Plan(Ng, 3, L, M, R=R) for Ng in sizes]
    cells = [synth.sample_mixture(synth.mixture_anisotropic(8400 + 10 * Ng + i, 3), Ng, L)
             for Ng, k in zip(sizes, counts) for i in range(k)]
    res = {}
    for mode in (E.EC_SCHED_TERMS, E.EC_SCHED_FUSED):
        b = E.Batch(plans, counts, E.EC_FP64)
        if mode == E.EC_SCHED_TERMS:
            assert [b.get_schedule(g)[0] for g in range(3)] == [E.EC_SCHED_TERMS] * 3
            b.set_schedule(0, E.EC_SCHED_TERMS, 2, 0)           # 3 cells in passes of 2
        else:
            for g, Ng in enumerate(sizes):       # the term-parallel default splits
                b.set_schedule(g, E.EC_SCHED_FUSED, 0, {16: 1, 24: 3, 32: 4}[Ng])
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.collide(f, Q)
        b.step(f, 0.01, 3, None)
        torch.cuda.synchronize()
        res[mode] = (E.unpack(b, Q.cpu().numpy()), E.unpack(b, f.cpu().numpy()))
        b.close()
    (qt, ft), (qf, ff) = res[E.EC_SCHED_TERMS], res[E.EC_SCHED_FUSED]
    ops = {Ng: efm.make_plan(Ng, 3, L, M, R=R) for Ng in sizes}
    for c in range(len(cells)):
        # scale: the gain at the 16 largest-F points (the oracle's); the two
        # schedules add the same products in the same order and differ only
        # where the fused kernel contracts a product into its sum
        Ng = cells[c].shape[0]
        _, qp, _, _ = efm.collide_points(ops[Ng], cells[c], np.argsort(cells[c].ravel())[-16:])
        dq = np.abs(qt[c] - qf[c]).max() / np.abs(qp).max()
        df = np.abs(ft[c] - ff[c]).max() / np.abs(ff[c]).max()
        say(f"  cell {c} ({Ng}^3): Q {dq:.2e} of the gain, 3 steps {df:.2e}")
        assert np.all(np.isfinite(qt[c])) and dq <= 1e-14 and df <= 1e-14


@pytest.mark.parametrize("Nl,prec,ncell", [(16, 0, 192), (24, 1, 80), (32, 0, 48)])
def test_terms_at_the_default_crossover(Nl, prec, ncell):
    """The largest groups that start on the term-parallel schedule (the
    measured crossover with the fused one): every cell against the fused
    schedule at the same x split, whose products and order of sums it
    shares (1e-13 of each
    cell's max |Q|: J = 33 products per point rounded apart from their sum,
    on gains up to ~20x |Q| for these mixtures), two cells against the
    oracle at sampled points."""
    import torch
    say(f"case term-parallel default at {ncell} cells of {Nl}^3 precision={prec}")
    plan = E.Plan(Nl, 3, L, M, R=R)
    base = [synth.sample_mixture(synth.mixture_anisotropic(8500 + Nl + i, 3), Nl, L)
            for i in range(8)]
    cells = [base[i % 8] * (1.0 + 1e-3 * i) for i in range(ncell)]
    out = {}
    for mode in (E.EC_SCHED_TERMS, E.EC_SCHED_FUSED):
        b = E.Batch([plan], [ncell], prec)
        if mode == E.EC_SCHED_TERMS:
            assert b.get_schedule(0)[0] == E.EC_SCHED_TERMS
        else:
            b.set_schedule(0, E.EC_SCHED_FUSED, 0, {16: 1, 24: 3, 32: 4}[Nl])   # same split
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.collide(f, Q)
        torch.cuda.synchronize()
        out[mode] = E.unpack(b, Q.cpu().numpy())
        b.close()
        del f, Q
    qt, qf = out[E.EC_SCHED_TERMS], out[E.EC_SCHED_FUSED]
    worst = max(np.abs(qt[c] - qf[c]).max() / np.abs(qf[c]).max() for c in range(ncell))
    say(f"  worst cell vs fused {worst:.2e}")
    assert all(np.all(np.isfinite(q)) for q in qt) and worst <= 1e-13
    op = efm.make_plan(Nl, 3, L, M, R=R)
    rng = np.random.default_rng(Nl)
    for c in (0, ncell - 1):
        idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-12:],
                                        rng.choice(Nl ** 3, 20, replace=False)]))
        q, qp, qm, _ = efm.collide_points(op, cells[c], idx)
        err = np.abs(qt[c].ravel()[idx] - q).max() / np.abs(qp).max()
        say(f"  cell {c} vs oracle {err:.2e}")
        assert err <= bound_pts(prec, Nl, 3, qp, qm)


@pytest.mark.parametrize("Nl,prec", [(16, 0), (32, 0), (32, 1)])
def test_terms_with_a_ragged_term_count(Nl, prec):
    """M = 13 directions: 13 gain terms, so the sum kernel's loads of 8 terms
    at a time leave 5; against the fused schedule at the same x split and
    the oracle."""
    import torch
    split = {16: 1, 32: 2}[Nl]
    say(f"case term-parallel {Nl}^3 M=13 precision={prec} split={split}")
    plan = E.Plan(Nl, 3, L, 13, R=R)
    cells = [synth.sample_mixture(synth.mixture_anisotropic(8600 + Nl + i, 3), Nl, L)
             for i in range(2)]
    out = {}
    for mode in (E.EC_SCHED_TERMS, E.EC_SCHED_FUSED):
        b = E.Batch([plan], [2], prec)
        b.set_schedule(0, mode, 0, split)
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.collide(f, Q)
        torch.cuda.synchronize()
        out[mode] = E.unpack(b, Q.cpu().numpy())
        b.close()
    op = efm.make_plan(Nl, 3, L, 13, R=R)
    rng = np.random.default_rng(13 + Nl)
    for c in range(2):
        qt, qf = out[E.EC_SCHED_TERMS][c], out[E.EC_SCHED_FUSED][c]
        idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-16:],
                                        rng.choice(Nl ** 3, 32, replace=False)]))
        q, qp, qm, _ = efm.collide_points(op, cells[c], idx)
        scale = np.abs(qp).max()
        d_fused = np.abs(qt - qf).max() / scale
        err = np.abs(qt.ravel()[idx] - q).max() / scale
        say(f"  cell {c}: vs fused {d_fused:.2e} of the gain, vs oracle {err:.2e}")
        assert np.all(np.isfinite(qt)) and d_fused <= 1e-14 and err <= bound_pts(prec, Nl, 3, qp, qm)


def _collide_2d(N, cells, prec):
    import torch
    p = E.Plan(N, 2, 8.0, 16, R=6.0)
    b = E.Batch([p], [len(cells)], prec)
    b.set_schedule(0, E.EC_SCHED_TERMS, 0, 0)
    f = to_dev(E.pack(b, cells))
    Q = torch.full_like(f, float("nan"))
    b.collide(f, Q)
    torch.cuda.synchronize()
    out = E.unpack(b, Q.cpu().numpy())
    b.close()
    return out


@pytest.mark.parametrize("N,prec,ncell", [(8, 0, 3), (8, 1, 2), (12, 0, 2), (12, 1, 2),
                                          (16, 0, 3), (16, 1, 2), (24, 1, 2), (32, 1, 2)])
def test_2d_one_block_per_cell(N, prec, ncell):
    """2D cells of the term-parallel schedule evaluated one block per cell
    (k_cell_2d: 17 groups of N threads for M' = 16, each transforming the
    cell and running one term, the products summed in LDS): every cell on the
    full grid against the oracle's double sum, within the stated bound."""
    from tests.gpu_util import bound_full, rel_err
    say(f"case 2D one block per cell N={N} precision={prec} cells={ncell}")
    cells = [synth.sample_mixture(synth.mixture_two_gaussians(8100 + N + c, 2), N, 8.0)
             for c in range(ncell)]
    out = _collide_2d(N, cells, prec)
    op = efm.make_plan(N, 2, 8.0, 16, R=6.0)
    for c in range(ncell):
        ref = efm.collide_modes(op, cells[c])
        err = rel_err(out[c], ref.Q, ref.Qplus)
        tol = bound_full(prec, N, 2, ref)
        say(f"  cell {c}: rel err {err:.3e} (bound {tol:.2e})")
        assert np.all(np.isfinite(out[c])) and err <= tol


def test_2d_one_block_switch_at_24():
    """At 24^2 FP64 the one-block kernel runs from 128 cells (below, the slab
    transform, the term kernel and the sum): batches of 127 and 128 cells
    agree on their common cells to 1e-13, and the first cell of the larger
    batch matches the oracle."""
    from tests.gpu_util import rel_err
    say("case 2D 24^2 FP64: 127 and 128 cells")
    cells = [synth.sample_mixture(synth.mixture_two_gaussians(8200 + c, 2), 24, 8.0)
             for c in range(128)]
    a = _collide_2d(24, cells[:127], 0)
    b = _collide_2d(24, cells, 0)
    for c in (0, 63, 126):
        d = np.linalg.norm(a[c] - b[c]) / np.linalg.norm(b[c])
        say(f"  cell {c}: |127 cells - 128 cells| / |Q| = {d:.3e}")
        assert d <= 1e-13
    ref = efm.collide_modes(efm.make_plan(24, 2, 8.0, 16, R=6.0), cells[0])
    err = rel_err(b[0], ref.Q, ref.Qplus)
    say(f"  cell 0 of 128 vs the oracle: {err:.3e}")
    assert np.all(np.isfinite(b[127])) and err <= 1e-12

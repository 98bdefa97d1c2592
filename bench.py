#!/usr/bin/env python3
"""Collision evaluations per second of the EFM operator on one MI355X.

Workload (the headline of the method: N = 32^3, M = 32): 3D hard-sphere
kernel, box [-8, 8]^3, R = 6, 32 hemisphere directions, a batch of 1024
independent cells, each a seeded sum of 2-4 anisotropic Gaussians (means
U[-2,2]^3, diagonal temperatures U[0.3,2], Dirichlet weights; seed 2001 + cell).
One step = one ec_collide over the whole batch (every cell's Q).  Inputs are
resident in HBM before the timed region.  FP64 is the headline value; FP32
transforms and single-cell latency are reported beside it, each with its
error against the CPU oracle on sampled points.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "collision evals/sec at N=32^3,M=32: FP64 vs mixed vs surrogate at stated rel err"
PEAK_FP64 = 78.6    # TFLOP/s, MI355X vector FP64
PEAK_FP32 = 157.3   # TFLOP/s, MI355X vector FP32
N, D, L, M, R = 32, 3, 8.0, 32, 6.0
KNAMES = ["k_fwd", "k_pencil", "k_slab", "k_pipe", "k_fwdx", "k_fused"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_flops(n_side: int, d: int, terms: int) -> list:
    """Algorithmic flops per cell of each kernel (nominal 2.5 n log2 n per real
    and 5 n log2 n per complex transform, split by axes passes; products and
    sums as written in the algorithm)."""
    n = n_side ** d
    lg = math.log2(n)
    if d == 3:
        fwd = (2.0 / 3.0) * 2.5 * n * lg
        pencil = (1.0 / 3.0) * 2.5 * n * lg + terms * (1.0 / 3.0) * 5.0 * n * lg \
            + (1.0 / 3.0) * 2.5 * n * lg + terms * 6.0 * n + 2.0 * n
        slab = terms * (2.0 / 3.0) * 5.0 * n * lg + (2.0 / 3.0) * 2.5 * n * lg \
            + terms * 2.0 * n + 2.0 * n
    else:
        fwd = 2.5 * n * lg
        pencil = 0.0
        slab = terms * 5.0 * n * lg + 2.5 * n * lg + terms * 8.0 * n + 4.0 * n
    total = fwd + pencil + slab
    # the fused schedule: k_fwd, then the x forward pass, then everything else
    fwdx = (1.0 / 3.0) * 2.5 * n * lg if d == 3 else 0.0
    return [fwd, pencil, slab, total, fwdx, total - fwd - fwdx]


def make_cells(n_cells, seed0=2001):
    import synth
    return [synth.sample_mixture(synth.mixture_anisotropic(seed0 + c, D), N, L) for c in range(n_cells)]


SCHED = {"mode": None, "chunk": 0, "G": 0}
TUNE_CACHE = os.path.join(ROOT, "paper_1704_07369_amd", "tune_cache.txt")


def time_collide(E, torch, plan, cells, precision, steps, warmup, profile):
    b = E.Batch([plan], [len(cells)], precision)
    if SCHED["mode"] is not None:
        b.set_schedule(0, SCHED["mode"], SCHED["chunk"], SCHED["G"])
    f = torch.from_numpy(E.pack(b, cells)).to("cuda:0")
    Q = torch.zeros_like(f)
    if SCHED["mode"] is None and len(cells) > 1:
        b.autotune(f, Q, TUNE_CACHE)
    for _ in range(warmup):
        b.collide(f, Q)
    torch.cuda.synchronize()
    if profile:
        b.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        b.collide(f, Q)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        ms, la, ce = b.profile_read()
        b.profile(False)
        prof = (ms[0], la[0], ce[0])
    log(f"bench: schedule {b.get_schedule(0)}")
    return b, f, Q, (t1 - t0), prof


def sampled_error(E, b, Q, cells, cell_ids, oplan, efm, npts=64):
    import numpy as np
    qh = E.unpack(b, Q.cpu().numpy())
    rng = np.random.default_rng(12345)
    worst = 0.0
    for c in cell_ids:
        # the points where F peaks are among the samples, so that max |Q+| over
        # the samples is the gain's scale
        idx = np.unique(np.concatenate([np.argsort(cells[c].ravel())[-16:],
                                        rng.choice(N ** D, npts, replace=False)]))
        q, qp, _, _ = efm.collide_points(oplan, cells[c], idx)
        worst = max(worst, float(np.abs(qh[c].ravel()[idx] - q).max() / np.abs(qp).max()))
    return worst


# HBM bytes per launch of the dominant kernels, 2 FETCH_SIZE + WRITE_SIZE (factors
# from the ec_copy calibration) of the run recorded in
# profiles/collide_n32_m32_default_counters.md; keyed by (kernel, precision,
# cells per launch) and valid for that code only (re-measure after changing it)
MEASURED_TRAFFIC = {
    ("k_fused", "f64", 1024): (2 * 2705696 + 262144) * 1024,
    ("k_fused", "f32", 512): (2 * 620835 + 131072) * 1024,
    ("k_pencil", "bf16x3", 1024): (2 * 236649 + 8650752) * 1024,
}


def roofline(prof, flops_cell, peak, prec="f64"):
    """Dominant kernel of the timed region: algorithmic flops it performed
    over its summed duration (HIP events on the launch stream)."""
    ms, launches, cells = prof
    k = max(range(len(ms)), key=lambda i: ms[i])
    fl = flops_cell[k]
    achieved = fl * cells / (ms[k] * 1e-3) / 1e12
    return {
        "bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": MEASURED_TRAFFIC.get((KNAMES[k], prec, round(cells / max(1, launches[k])))),
        "kernel": KNAMES[k],
        "avg_launch_ms": round(ms[k] / max(1, launches[k]), 5),
        "launches": int(launches[k]), "cells_per_launch": cells / max(1, launches[k]),
        "flops_per_launch": fl * cells / max(1, launches[k]),
        "kernel_ms_total": {KNAMES[i]: round(float(ms[i]), 3) for i in range(len(ms))},
    }


def relaxation_leg(E, torch, steps=200, dt=0.01, n_cells=4096, seed=3000):
    """Batched space-homogeneous relaxation: n_cells cells with grids mixed
    16^3/24^3/32^3 (40/35/25 %, seeded permutation), hard spheres, M = 32,
    FP64, `steps` forward-Euler steps replayed from one captured HIP graph,
    per-cell (mass, eta) after every step."""
    import numpy as np
    import synth
    sizes = synth.batch_mixed_sizes(seed, n_cells)
    groups = [16, 24, 32]
    plans = [E.Plan(Ng, D, L, M, R=R) for Ng in groups]
    counts = [int((sizes == Ng).sum()) for Ng in groups]
    order = [c for Ng in groups for c in np.nonzero(sizes == Ng)[0]]
    cells = [synth.sample_mixture(synth.mixture_anisotropic(3001 + int(c), D), int(sizes[c]), L)
             for c in order]
    b = E.Batch(plans, counts, E.EC_FP64)
    f = torch.from_numpy(E.pack(b, cells)).to("cuda:0")
    Q = torch.zeros_like(f)
    b.autotune(f, Q, TUNE_CACHE)
    mon = torch.zeros(steps * n_cells * 2, dtype=torch.float64, device="cuda:0")
    b.step(f, dt, 1, mon)          # graph capture + warm-up
    f.copy_(torch.from_numpy(E.pack(b, cells)).to("cuda:0"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(f, dt, steps, mon)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    m = mon.view(steps, n_cells, 2).cpu().numpy()
    mass_drift = float(np.max(np.abs(m[-1, :, 0] - m[0, :, 0]) / m[0, :, 0]))
    deta = np.diff(m[:, :, 1], axis=0)
    fmin = float(f.min().item())
    return {"workload": f"{n_cells} cells mixed 16^3/24^3/32^3 ({counts}), hard sphere, M=32, "
                        f"FP64, {steps} forward-Euler steps dt={dt} in one HIP graph",
            "seconds": t, "cell_evals_per_s": n_cells * steps / t, "ms_per_step": t / steps * 1e3,
            "max_rel_mass_drift": mass_drift, "max_eta_increase": float(deta.max()),
            "min_F": fmin}


def surrogate_leg(E, torch, seconds=40.0, n_traj=500, n_steps=100, n_test=1024, dt=0.01, log_fn=None):
    """Learned surrogate at the headline size: (F, Q) pairs from n_traj
    forward-Euler trajectories of the exact FP64 operator (seeds 5001 + i,
    n_steps steps each), training by the library's own kernels for `seconds`,
    then n_test fresh cells (seeds 6001 + i): relative L2 error of the raw
    network and of the screened result against the FP64 operator, fallback
    count, and evals/s of the screened path (network, screen and fallback
    inside the timed region) beside the exact operator's."""
    import numpy as np
    import synth
    from paper_1704_07369_amd.surrogate import DEFAULT, Surrogate, generate_pairs, train
    plan = E.Plan(N, D, L, M, R=R)
    sur = Surrogate(N, seed=1234, max_batch=64, **DEFAULT)
    t0 = time.perf_counter()
    cells = [synth.sample_mixture(synth.mixture_anisotropic(5001 + i, D), N, L) for i in range(n_traj)]
    Fin, Tgt = generate_pairs(torch, plan, cells, n_steps, dt, sur)
    t_gen = time.perf_counter() - t0
    del cells
    hist, steps = train(torch, sur, Fin, Tgt, seconds=seconds, batch=16, lr=2e-3, log=log_fn)
    npairs = int(Fin.shape[0])
    del Fin, Tgt
    torch.cuda.empty_cache()
    test = [synth.sample_mixture(synth.mixture_anisotropic(6001 + i, D), N, L) for i in range(n_test)]
    b = E.Batch([plan], [n_test], E.EC_FP64)
    f = torch.from_numpy(E.pack(b, test)).to("cuda:0")
    Qe = torch.zeros_like(f)
    b.autotune(f, Qe, TUNE_CACHE)
    b.collide(f, Qe)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b.collide(f, Qe)
    torch.cuda.synchronize()
    t_exact = (time.perf_counter() - t0) / 3
    # raw network output (no screen), per-cell relative L2 error
    n = N ** D
    mb = sur.max_batch
    xin = torch.empty((mb, n), dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(xin)
    Qr = torch.empty((n_test, n), dtype=torch.float64, device="cuda:0")
    h3 = (2 * L / N) ** 3
    c0 = (2 * math.pi) ** 1.5
    fv = f.view(n_test, n)
    for c in range(0, n_test, mb):
        k = min(mb, n_test - c)
        sur.prepare(b, f, None, c, k, xin[:k], None)
        sur.forward(xin[:k], y[:k], k)
        mass = h3 * fv[c:c + k].sum(1, keepdim=True)
        Qr[c:c + k] = y[:k].double() * mass ** 2 / c0 ** 2
    Qev = Qe.view(n_test, n)
    raw = ((Qr - Qev).norm(dim=1) / Qev.norm(dim=1)).cpu().numpy()
    Qs = torch.zeros_like(f)
    fell = torch.zeros(n_test, dtype=torch.int32, device="cuda:0")
    sur.collide(b, f, Qs, tau_m=-1.0, fell_back=fell)       # screen off: projected network
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        sur.collide(b, f, Qs, tau_m=-1.0, fell_back=fell)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t0) / 3
    proj = ((Qs.view(n_test, n) - Qev).norm(dim=1) / Qev.norm(dim=1)).cpu().numpy()
    scr_d = torch.zeros(n_test * 4, dtype=torch.float64, device="cuda:0")
    sur.collide(b, f, Qs, tau_m=-1.0, fell_back=fell, screen=scr_d)
    scr_h = scr_d.view(n_test, 4).cpu().numpy()
    sweep = []
    for tm, te in [(1e-3, 1e-2), (1e-2, 1e-2), (1e-2, 5e-2), (5e-2, 5e-2), (1.0, 1.0)]:
        ok = (scr_h[:, 0] <= 0) & (scr_h[:, 1] <= tm) & (scr_h[:, 2] <= te) & (scr_h[:, 3] <= te)
        sweep.append({"tau_m": tm, "tau_e": te, "accepted": int(ok.sum()),
                      "accepted_rel_l2_max": float(proj[ok].max()) if ok.any() else None})
    nf = sur.collide(b, f, Qs, fell_back=fell)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        nf = sur.collide(b, f, Qs, fell_back=fell)
    torch.cuda.synchronize()
    t_sur = (time.perf_counter() - t0) / 3
    scr = ((Qs.view(n_test, n) - Qev).norm(dim=1) / Qev.norm(dim=1)).cpu().numpy()
    acc = fell.cpu().numpy() == 0
    return {
        "workload": f"FNO {DEFAULT['layers']} layers x {DEFAULT['channels']} channels x "
                    f"{DEFAULT['modes']} modes, FP32, trained {seconds:.0f} s on {npairs} pairs "
                    f"({n_traj} FE trajectories x {n_steps} steps of the FP64 operator), "
                    f"tested on {n_test} fresh cells",
        "train_steps": steps, "train_batch": 16, "data_gen_s": round(t_gen, 2),
        "final_train_loss": hist[-1][2] if hist else None,
        "raw_rel_l2_median": float(np.median(raw)), "raw_rel_l2_max": float(raw.max()),
        "projected_rel_l2_median": float(np.median(proj)), "projected_rel_l2_max": float(proj.max()),
        "projected_evals_per_s": n_test / t_net,
        "screen_sweep": sweep,
        "raw_residual_median": [float(np.median(scr_h[:, i])) for i in (1, 2, 3)],
        "fallback_cells": int(nf),
        "accepted_rel_l2_median": float(np.median(scr[acc])) if acc.any() else None,
        "accepted_rel_l2_max": float(scr[acc].max()) if acc.any() else None,
        "screened_rel_l2_max": float(scr.max()),
        "screened_evals_per_s": n_test / t_sur, "exact_fp64_evals_per_s": n_test / t_exact,
        "gain_vs_exact_fp64": t_exact / t_sur,
    }


def precision_sweep_leg(E, torch, n_cells=256, reps=2):
    """Precision sweep on the non-separable kernel: 3D variable hard spheres
    (gamma = 0.5), N = 64^3, M = 64 directions x 8 radial nodes (513
    transforms per evaluation), n_cells two-Gaussian mixtures (means
    U[-2,2]^3, temperatures U[0.5,1.5], seed 4001 + cell).  FP64, FP32 and
    split-BF16 evaluations timed; FP32 and split-BF16 errors against the FP64
    GPU result on every cell (the FP64 path itself is checked against the
    oracle at 64^3 in the GPU tests; the oracle's tables at this size are out
    of reach of a bench run)."""
    import numpy as np
    import synth
    Nn, Mm, nr, gam = 64, 64, 8, 0.5
    t0 = time.perf_counter()
    plan = E.Plan(Nn, D, L, Mm, kind=E.EC_KERNEL_VHS, R=R, gamma=gam, n_radial=nr)
    t_plan = time.perf_counter() - t0
    cells = [synth.sample_mixture(synth.mixture_two_gaussians(4001 + c, D), Nn, L) for c in range(n_cells)]
    out = {"workload": f"3D VHS gamma={gam}, N=64^3, M={Mm} x {nr} radial = {plan.terms()} products, "
                       f"{n_cells} two-Gaussian cells", "plan_setup_s": round(t_plan, 2)}
    Qs, P = {}, {}
    for prec, name in ((E.EC_FP64, "fp64"), (E.EC_FP32, "fp32"), (E.EC_BF16X3, "bf16x3")):
        b = E.Batch([plan], [n_cells], prec)
        f = torch.from_numpy(E.pack(b, cells)).to("cuda:0")
        Q = torch.zeros_like(f)
        b.collide(f, Q)                       # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.collide(f, Q)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        ep = torch.zeros(n_cells, dtype=torch.float64, device="cuda:0")
        b.entropy_prod(f, Q, ep)
        torch.cuda.synchronize()
        Qs[name] = torch.stack([Q[int(o):int(o) + Nn ** 3] for o in b.offsets])
        P[name] = ep.cpu().numpy()
        out[name] = {"evals_per_s": n_cells / t, "ms_per_eval_batch": t * 1e3,
                     "schedule": list(b.get_schedule(0))}
        log(f"bench: sweep {name} {n_cells / t:.4g} evals/s")
        del b, f, Q
    q64 = Qs["fp64"]
    for name in ("fp32", "bf16x3"):
        d = (Qs[name] - q64).view(n_cells, -1).norm(dim=1) / q64.view(n_cells, -1).norm(dim=1)
        d = d.cpu().numpy()
        pe = np.abs(P[name] - P["fp64"]) / np.abs(P["fp64"])
        out[name].update({"rel_l2_vs_fp64_median": float(np.median(d)), "rel_l2_vs_fp64_max": float(d.max()),
                          "entropy_prod_rel_err_max": float(pe.max())})
    return out


def cpu_baseline(cells, efm, oplan, budget_s=10.0):
    """The oracle (plain double sum over modes, OpenMP over all host threads)
    on as many cells of the workload as fit in about budget_s seconds (at
    least one); evals/s = cells / time.  Beside it, the same fast algorithm
    the library runs (one forward and M'+1 packed inverse FFTs per cell, on
    the oracle's tables, torch FP64 FFTs on the host threads): a like-for-like
    CPU rate for the transform-based method."""
    import numpy as np
    import torch
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    efm._load()
    t0 = time.perf_counter()
    done = 0
    ref0 = None
    while done < len(cells) and (done == 0 or time.perf_counter() - t0 < budget_s):
        ref = efm.collide_modes(oplan, cells[done])
        ref0 = ref0 or ref
        done += 1
    t = time.perf_counter() - t0
    out = {"value": done / t, "unit": "evals/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} of the 1024 cells, full 32^3 direct double sum over modes (M=32), "
                     f"{t:.1f} s"}
    # fast algorithm on the host
    torch.set_num_threads(threads)
    shp = (N,) * D
    lr, sig = oplan.lr, oplan.sigma
    G = torch.from_numpy(((lr.c[:, None] * sig * lr.U) + 1j * (sig * lr.V)).reshape((-1,) + shp))
    Dg = torch.from_numpy((sig * sig * lr.diagonal()).reshape(shp)).to(torch.complex128)
    t0 = time.perf_counter()
    k = 0
    while k < len(cells) and (k == 0 or time.perf_counter() - t0 < 0.5 * budget_s):
        F = torch.from_numpy(cells[k])
        Fh = torch.fft.fftn(F.to(torch.complex128))
        qp = torch.zeros(shp, dtype=torch.float64)
        for j in range(G.shape[0]):
            c = torch.fft.ifftn(G[j] * Fh)
            qp += c.real * c.imag
        q = qp - F * torch.fft.ifftn(Dg * Fh).real
        if k == 0:
            err = float(np.abs(q.numpy() - ref0.Q).max() / np.abs(ref0.Qplus).max())
        k += 1
    t = time.perf_counter() - t0
    out["fast_fft_cpu"] = {"value": k / t, "unit": "evals/s", "cores": threads,
                           "sample": f"{k} cells, torch FP64 FFTs, {t:.1f} s",
                           "max_err_vs_oracle": err}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cells", type=int, default=1024)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the oracle timing")
    ap.add_argument("--skip-parity", action="store_true")
    ap.add_argument("--skip-fp32", action="store_true", help="omit the FP32 side (profiling runs)")
    ap.add_argument("--skip-single", action="store_true", help="omit single-cell latency")
    ap.add_argument("--schedule", choices=["auto", "pipeline", "two_pass", "fused"], default="auto")
    ap.add_argument("--chunk", type=int, default=0, help="cells per pass/chunk (0 = default)")
    ap.add_argument("--term-groups", type=int, default=0)
    ap.add_argument("--skip-relax", action="store_true", help="omit the mixed-N relaxation leg")
    ap.add_argument("--skip-surrogate", action="store_true", help="omit the learned-surrogate leg")
    ap.add_argument("--skip-sweep", action="store_true", help="omit the 64^3 VHS precision sweep")
    ap.add_argument("--surrogate-seconds", type=float, default=40.0, help="surrogate training budget")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run ec_copy on a buffer of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): cells are independent "
              "and would be split across GPUs by cost with no exchange per step, but that "
              "split is not implemented or measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch
    import paper_1704_07369_amd as E

    assert torch.cuda.is_available(), "no GPU"
    if args.schedule != "auto":
        SCHED["mode"] = {"pipeline": E.EC_SCHED_PIPELINE, "two_pass": E.EC_SCHED_TWO_PASS,
                         "fused": E.EC_SCHED_FUSED}[args.schedule]
        SCHED["chunk"], SCHED["G"] = args.chunk, args.term_groups
    if args.copy_mb:
        nc = args.copy_mb * 1048576 // 8
        a = torch.ones(nc, dtype=torch.float64, device="cuda:0")
        bb = torch.zeros_like(a)
        for _ in range(3):
            E.ec_copy(a, bb, nc)
        torch.cuda.synchronize()
        log(f"bench: ec_copy of {args.copy_mb} MiB x3 done (16 n bytes each)")
        del a, bb
    log(f"bench: building {args.cells} cells of {N}^3")
    cells = make_cells(args.cells)
    plan = E.Plan(N, D, L, M, R=R)
    terms = plan.terms()
    flops = kernel_flops(N, D, terms)
    flops_eval = flops[3]

    log("bench: FP64 timed region")
    b64, f64, Q64, t64, prof64 = time_collide(E, torch, plan, cells, E.EC_FP64, args.steps,
                                              args.warmup, True)
    ev64 = args.cells * args.steps / t64
    log(f"bench: FP64 {ev64:.4g} evals/s")
    ev32 = t32 = prof32 = b32 = Q32 = None
    if not args.skip_fp32:
        log("bench: FP32 timed region")
        b32, f32, Q32, t32, prof32 = time_collide(E, torch, plan, cells, E.EC_FP32, args.steps,
                                                  args.warmup, True)
        ev32 = args.cells * args.steps / t32
        log(f"bench: FP32 {ev32:.4g} evals/s")
    evb = tb = profb = bb = Qb = None
    if not args.skip_fp32:
        log("bench: split-BF16 MFMA x pass timed region")
        bb, fb, Qb, tb, profb = time_collide(E, torch, plan, cells, E.EC_BF16X3, args.steps,
                                             args.warmup, True)
        evb = args.cells * args.steps / tb
        log(f"bench: BF16x3 {evb:.4g} evals/s")
    t1_64 = t1_32 = None
    reps = max(10, args.steps)
    if not args.skip_single:
        log("bench: single-cell latency")
        one = cells[:1]
        _, _, _, t1_64, _ = time_collide(E, torch, plan, one, E.EC_FP64, reps, 2, False)
        _, _, _, t1_32, _ = time_collide(E, torch, plan, one, E.EC_FP32, reps, 2, False)
        import synth
        small_us = {}
        for Ns in (16, 24):       # one cell of the smaller grids of the mixed-N leg
            ps = E.Plan(Ns, D, L, M, R=R)
            one_s = [synth.sample_mixture(synth.mixture_anisotropic(2001, D), Ns, L)]
            bs, _, _, ts, _ = time_collide(E, torch, ps, one_s, E.EC_FP64, reps, 2, False)
            small_us[f"n{Ns}_fp64_us"] = ts / reps * 1e6
            bs.close()

    out = {
        "metric": METRIC, "value": ev64, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t64 / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D hard-sphere EFM collision operator, N=32^3, M=32 directions, "
                               f"L=8, R=6, batch of {args.cells} Gaussian-mixture cells, FP64",
                   "d": D, "N": N, "M": M, "L": L, "R": R, "cells": args.cells,
                   "kernel": "hard_sphere", "flops_per_eval": flops_eval},
        "roofline": roofline(prof64, flops, PEAK_FP64),
    }
    if ev32 is not None:
        out["fp32"] = {"value": ev32, "ms_per_step": t32 / args.steps * 1e3,
                       "roofline": roofline(prof32, flops, PEAK_FP32, "f32")}
    if evb is not None:
        out["bf16x3"] = {"value": evb, "ms_per_step": tb / args.steps * 1e3,
                         "roofline": roofline(profb, flops, PEAK_FP32, "bf16x3")}
    if t1_64 is not None:
        out["single_cell"] = {"fp64_us": t1_64 / reps * 1e6, "fp32_us": t1_32 / reps * 1e6,
                              **small_us}
    # the device as it runs: vector FMA throughput measured by ec_valu_probe,
    # beside the published peaks that `roofline.peak` uses
    log("bench: vector-ALU probe")
    meas64 = E.ec_valu_probe(E.EC_FP64)
    out["roofline"]["measured_peak"] = round(meas64, 2)
    out["roofline"]["frac_of_measured"] = round(out["roofline"]["achieved"] / meas64, 4)
    if ev32 is not None:
        meas32 = E.ec_valu_probe(E.EC_FP32)
        r32 = out["fp32"]["roofline"]
        r32["measured_peak_unpacked"] = round(meas32, 2)
        r32["frac_of_measured_unpacked"] = round(r32["achieved"] / meas32, 4)
    if not args.skip_relax:
        log("bench: mixed-N relaxation leg (200 graph-replayed FE steps)")
        out["relaxation"] = relaxation_leg(E, torch)
    if not args.skip_sweep:
        log("bench: 64^3 VHS precision sweep")
        out["precision_sweep"] = precision_sweep_leg(E, torch)
    if not args.skip_surrogate:
        log("bench: learned surrogate (data, training, screened inference)")
        out["surrogate"] = surrogate_leg(E, torch, seconds=args.surrogate_seconds, log_fn=log)
        log(f"bench: surrogate {out['surrogate']}")
    if not args.skip_parity or not args.skip_cpu:
        from oracle import efm
        log("bench: oracle tables (quadrature)")
        oplan = efm.make_plan(N, D, L, M, R=R)
        if not args.skip_parity:
            log("bench: sampled parity vs oracle")
            out["parity"] = {
                "metric": "max_r |Q - Q_oracle| / max_r |Q+_oracle| on 64 random and the 16 largest-F points x 2 cells",
                "fp64": sampled_error(E, b64, Q64, cells, [0, args.cells - 1], oplan, efm),
            }
            if b32 is not None:
                out["parity"]["fp32"] = sampled_error(E, b32, Q32, cells, [0, args.cells - 1],
                                                      oplan, efm)
            if bb is not None:
                out["parity"]["bf16x3"] = sampled_error(E, bb, Qb, cells, [0, args.cells - 1],
                                                        oplan, efm)
            # every cell of the batch against the FP64 GPU result
            n = N ** D
            if Q64.numel() == args.cells * n:
                ref = Q64.view(args.cells, n)
                den = torch.linalg.vector_norm(ref, dim=1)
                for name, Qp in (("fp32", Q32), ("bf16x3", Qb)):
                    if Qp is None or Qp.numel() != Q64.numel():
                        continue
                    r = torch.linalg.vector_norm(Qp.view(args.cells, n) - ref, dim=1) / den
                    out["parity"][f"{name}_vs_fp64_gpu_all_cells"] = {
                        "metric": "per-cell ||Q - Q_fp64|| / ||Q_fp64|| over all cells",
                        "median": float(r.median()), "max": float(r.max())}
        if not args.skip_cpu:
            log("bench: CPU baseline (oracle)")
            out["cpu_baseline"] = cpu_baseline(cells, efm, oplan)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

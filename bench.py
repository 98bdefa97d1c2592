#!/usr/bin/env python3
"""Collision evaluations per second of the EFM operator on one MI355X.

Workload (the headline of the method: N = 32^3, M = 32): 3D hard-sphere
kernel, box [-8, 8]^3, R = 6, 32 hemisphere directions, a batch of 1024
independent cells, each a seeded sum of 2-4 anisotropic Gaussians (means
U[-2,2]^3, diagonal temperatures U[0.3,2], Dirichlet weights; seed 2001 + cell).
One step = one ec_collide over the whole batch (every cell's Q).  Inputs are
resident in HBM before the timed region.  FP64 is the headline value; FP32
transforms, the split-BF16 x pass and single-cell latency (3D and the 2D
32^2, M = 16 configuration) are reported beside it.  Roofline: algorithmic
flops (nominal FFT convention) of the dominant kernel over its duration from
HIP events on the launch stream in the timed region; HBM bytes per launch
from rocprofv3 byte counters of a child run of the same batches, calibrated
by a plain copy.  Parity: the full grid of 8 cells against the oracle's
double sum (the same oracle runs are the CPU baseline), each path against
its stated bound.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import math
import os
import shutil
import signal
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "collision evals/sec at N=32^3,M=32: FP64 vs mixed vs surrogate at stated rel err"
PEAK_FP64 = 78.6    # TFLOP/s, MI355X vector FP64
PEAK_FP32 = 157.3   # TFLOP/s, MI355X vector FP32
PEAK_BF16_MFMA = 2500.0   # TFLOP/s, MI355X dense BF16 matrix cores
COPY_MIB = 256            # ec_copy size of the byte-counter calibration
FULL_GRID_CELLS = [0, 127, 128, 255, 256, 511, 512, 1023]   # pass and round boundaries
N, D, L, M, R = 32, 3, 8.0, 32, 6.0
KNAMES = ["k_fwd", "k_pencil", "k_slab", "k_pipe", "reserved", "k_fused"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def flops_8d(n_side: int, d: int, terms: int) -> float:
    """Algorithmic flops of one collision evaluation in the nominal FFT
    convention (2.5 n log2 n per real transform): (2M'+2) 2.5 n log2 n for
    the forward and the 2M'+1 real inverse transforms, M'(4H + 3n) for the
    spectral multiplies and the weighted products, 2H + 2n for the loss
    (H = N^{d-1} (N/2 + 1) half-spectrum entries, n = N^d).  86.58 MFLOP at
    32^3, M' = 32; 12.78 GFLOP at 64^3, M' = 512."""
    n = n_side ** d
    H = n_side ** (d - 1) * (n_side // 2 + 1)
    lg = math.log2(n)
    return (2 * terms + 2) * 2.5 * n * lg + terms * (4 * H + 3 * n) + 2 * H + 2 * n


def kernel_flops(n_side: int, d: int, terms: int) -> list:
    """The same work split over the kernels that do it, indexed like the
    profile slots (k_fwd, k_pencil, k_slab, k_pipe, reserved, k_fused): in 3D
    the two-pass schedule's slab transform does the forward transform's y, z
    passes (2/3), its x pass (forward x, the inverse x passes, the
    multiplies) and slab pass (inverse y, z passes, products, loss) the rest;
    the fused schedules' forward kernel (slot 0 there) does the whole forward
    transform, their fused kernel everything after it; the pipelined kernel
    does all of it."""
    n = n_side ** d
    H = n_side ** (d - 1) * (n_side // 2 + 1)
    lg = math.log2(n)
    fwd = 2.5 * n * lg
    inv = (2 * terms + 1) * 2.5 * n * lg
    total = flops_8d(n_side, d, terms)
    if d == 3:
        k_fwd = fwd * 2 / 3
        k_pencil = fwd / 3 + inv / 3 + terms * 4 * H + 2 * H
        k_slab = inv * 2 / 3 + terms * 3 * n + 2 * n
    else:
        k_fwd = fwd
        k_pencil = 0.0
        k_slab = total - fwd
    return [k_fwd, k_pencil, k_slab, total, 0.0, total - fwd]


def bf16_gemm_flops(n_side: int, d: int, terms: int) -> float:
    """Matrix-core flops of the split-BF16 x pass per cell: for every pencil
    and each of the J = M'+1 inverse transforms, a (2N x 2N) real DFT matrix
    times a 2N vector, three products (hi hi, hi lo, lo hi)."""
    pencils = n_side ** (d - 1)
    return 3 * 2 * (2 * n_side) ** 2 * pencils * (terms + 1)


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


def roofline(prof, flops_cell, peak, traffic=None, bound="alu", unit="TFLOP/s"):
    """Dominant kernel of the timed region: its algorithmic flops (the
    per-kernel split of flops_8d, or the GEMM flops of a matrix-core stage)
    over its summed duration, from HIP events the library records on the
    launch stream around every launch.  traffic: HBM bytes per launch from
    the byte counters of the same kernel and workload (measure_traffic), or
    None."""
    ms, launches, cells = prof
    k = max(range(len(ms)), key=lambda i: ms[i])
    fl = flops_cell[k]
    achieved = fl * cells / (ms[k] * 1e-3) / 1e12
    nl = max(1, int(launches[k]))
    return {
        "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": traffic,
        "kernel": KNAMES[k],
        "avg_launch_ms": round(ms[k] / nl, 5),
        "launches": int(launches[k]), "cells_per_launch": cells / nl,
        "flops_per_cell": fl, "flops_per_launch": fl * cells / nl,
        "kernel_ms_total": {KNAMES[i]: round(float(ms[i]), 3) for i in range(len(ms))},
    }


# ---------------------------------------------------------------------------
# HBM bytes per launch from hardware counters: bench.py re-runs itself as a
# child under rocprofv3 --pmc (FETCH_SIZE, then WRITE_SIZE: they do not fit one
# pass), running the same batches with the same schedules plus a plain copy
# of known size that calibrates each counter to bytes.
# ---------------------------------------------------------------------------

COUNTER_KERNELS = {            # (profile slot, precision) -> kernel-name pattern
    ("k_fused", "f64"): ("k_fused", "<double"),
    ("k_fused", "f32"): ("k_fused", "<float"),
    ("k_pencil", "bf16x3"): ("k_pencil_bf16", ""),
}


def counter_child(args):
    """Runs under rocprofv3: the copy, then the FP64, FP32 and split-BF16
    batches of the timed regions (schedules from the tune cache), twice each."""
    import torch
    import paper_1704_07369_amd as E
    nc = COPY_MIB * 1048576 // 8
    a = torch.ones(nc, dtype=torch.float64, device="cuda:0")
    bb = torch.zeros_like(a)
    for _ in range(2):
        E.ec_copy(a, bb, nc)
    torch.cuda.synchronize()
    del a, bb
    cells = make_cells(args.cells)
    plan = E.Plan(N, D, L, M, R=R)
    for prec in (E.EC_FP64, E.EC_FP32, E.EC_BF16X3):
        b = E.Batch([plan], [len(cells)], prec)
        f = torch.from_numpy(E.pack(b, cells)).to("cuda:0")
        Q = torch.zeros_like(f)
        b.autotune(f, Q, TUNE_CACHE)
        for _ in range(2):
            b.collide(f, Q)
        torch.cuda.synchronize()
        log(f"bench counter child: precision {prec} done")
        b.close()
        del f, Q


def _read_counter_csv(d):
    """{kernel name: [counter value per dispatch]} from rocprofv3's CSV."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection*.csv"), recursive=True)
    per = {}
    for fn in files:
        with open(fn, newline="") as fh:
            for row in csv.DictReader(fh):
                key = (row.get("Dispatch_Id") or row.get("Correlation_Id"), row.get("Kernel_Name", ""))
                per[key] = per.get(key, 0.0) + float(row.get("Counter_Value") or 0.0)
    out = {}
    for (_, name), v in per.items():
        out.setdefault(name, []).append(v)
    return out


def _reap_group(pgid, what):
    """End whatever is left of a finished child's own session (the profiler
    can leave a helper behind when it exits), so that the bench leaves no
    process running."""
    try:
        os.killpg(pgid, 0)
    except (ProcessLookupError, PermissionError):
        return
    log(f"bench: {what} run left processes in its group; ending them")
    try:
        os.killpg(pgid, signal.SIGKILL)
    except ProcessLookupError:
        pass


def measure_traffic(args):
    """HBM bytes per launch of the dominant kernels, 2 counter runs of the
    child; None where rocprofv3 is missing or a run fails."""
    exe = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(exe):
        return None, "rocprofv3 not found"
    vals = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        d = tempfile.mkdtemp(prefix="efm_pmc_", dir="/tmp")
        cmd = [exe, "--pmc", ctr, "-d", d, "-o", "run", "--output-format", "csv", "--",
               sys.executable, os.path.abspath(__file__), "--counter-child", "--cells",
               str(args.cells)]
        log(f"bench: byte counter run {ctr}")
        with open(os.path.join(d, "rocprof.log"), "w") as lf:
            p = subprocess.Popen(cmd, cwd="/tmp", env=dict(os.environ, TMPDIR="/tmp"),
                                 stdout=lf, stderr=subprocess.STDOUT, start_new_session=True)
            try:
                rc = p.wait(timeout=240)
            except subprocess.TimeoutExpired:
                os.killpg(p.pid, signal.SIGKILL)
                p.wait()
                shutil.rmtree(d, ignore_errors=True)
                return None, f"{ctr} counter run timed out"
            _reap_group(p.pid, ctr)
        vals[ctr] = _read_counter_csv(d)
        shutil.rmtree(d, ignore_errors=True)
        # rocprofv3 can end with a signal after the program finished and the
        # results are complete; the CSV decides
        if not vals[ctr]:
            return None, f"{ctr} counter run gave no data (rc {rc})"

    def med(ctr, pat, prec_pat):
        xs = [v for name, vs in vals[ctr].items() if pat in name and prec_pat in name for v in vs]
        xs.sort()
        return xs[len(xs) // 2] if xs else None

    copy_kib = COPY_MIB * 1024.0          # bytes read = bytes written = 256 MiB
    cf, cw = med("FETCH_SIZE", "k_copy", ""), med("WRITE_SIZE", "k_copy", "")
    if not cf or not cw:
        return None, "no k_copy dispatch in the counter data"
    ff, fw = copy_kib / cf, copy_kib / cw
    out = {"calibration": {"copy_mib": COPY_MIB, "fetch_size_kib": cf, "write_size_kib": cw,
                           "fetch_factor": round(ff, 4), "write_factor": round(fw, 4)}}
    for key, (pat, pp) in COUNTER_KERNELS.items():
        fk, wk = med("FETCH_SIZE", pat, pp), med("WRITE_SIZE", pat, pp)
        if fk is None or wk is None:
            continue
        out[f"{key[0]}/{key[1]}"] = {"fetch_size_kib": fk, "write_size_kib": wk,
                                     "bytes": int(round(1024.0 * (ff * fk + fw * wk)))}
    return out, None


def relaxation_leg(E, torch, steps=200, dt=0.01, n_cells=4096, seed=3000):
    """Batched space-homogeneous relaxation: n_cells cells with grids mixed
    16^3/24^3/32^3 (40/35/25 %, seeded permutation), hard spheres, M = 32,
    FP64, `steps` forward-Euler steps launched as one captured HIP graph that
    holds every step (ec_step_graph), per-cell (mass, eta) after every step.
    The timed run reuses the graph of an untimed first run."""
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
    # capture of the graph that holds all the steps, and a warm-up run of it
    b.step(f, dt, steps, mon)
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


def surrogate_leg(E, torch, seconds=40.0, n_traj=5000, n_steps=10, n_test=1024, dt=0.01, log_fn=None):
    """Learned surrogate at the headline size: (F, Q) pairs from n_traj
    forward-Euler trajectories of the exact FP64 operator (seeds 5001 + i,
    n_steps steps each: 50 000 pairs, the fresh cells and their first steps,
    the distribution the surrogate is applied to), training by the library's
    own kernels for `seconds`, then n_test fresh cells (seeds 6001 + i):
    relative L2 error of the raw network and of the screened result against
    the FP64 operator, the stated bound and whether the accepted cells meet
    it, fallback count, and evals/s of the screened path (network, screen and
    fallback inside the timed region) beside the exact FP64 and FP32
    operator's."""
    import numpy as np
    import synth
    from paper_1704_07369_amd.surrogate import (DEFAULT, SCREEN_TAU_E, SCREEN_TAU_M,
                                                SURROGATE_BOUND, Surrogate, generate_pairs, train)
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
    b32 = E.Batch([plan], [n_test], E.EC_FP32)
    Q32 = torch.zeros_like(f)
    b32.autotune(f, Q32, TUNE_CACHE)
    b32.collide(f, Q32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        b32.collide(f, Q32)
    torch.cuda.synchronize()
    t_exact32 = (time.perf_counter() - t0) / 3
    e32 = ((Q32 - Qe).view(n_test, -1).norm(dim=1) / Qe.view(n_test, -1).norm(dim=1)).max().item()
    b32.close()
    del Q32
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
    for tm, te in [(SCREEN_TAU_M, SCREEN_TAU_E), (1e-3, -1.0), (1e-2, -1.0), (1e-3, 1e-2),
                   (1e-2, 5e-2), (1.0, -1.0)]:
        ok = (scr_h[:, 0] <= 0) & (scr_h[:, 1] <= tm)
        if te >= 0:
            ok &= (scr_h[:, 2] <= te) & (scr_h[:, 3] <= te)
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
        "screen": {"tau_m": SCREEN_TAU_M, "tau_e": SCREEN_TAU_E,
                   "rule": "H-functional of the projected Q <= 0 and raw mass residual <= tau_m"},
        "bound": SURROGATE_BOUND,
        "fallback_cells": int(nf),
        "accepted_rel_l2_median": float(np.median(scr[acc])) if acc.any() else None,
        "accepted_rel_l2_max": float(scr[acc].max()) if acc.any() else None,
        "within_bound": bool(scr.max() <= SURROGATE_BOUND),
        "screened_rel_l2_max": float(scr.max()),
        "screened_evals_per_s": n_test / t_sur, "exact_fp64_evals_per_s": n_test / t_exact,
        "exact_fp32_evals_per_s": n_test / t_exact32, "exact_fp32_rel_l2_max": e32,
        "gain_vs_exact_fp64": t_exact / t_sur, "gain_vs_exact_fp32": t_exact32 / t_sur,
    }


def precision_sweep_leg(E, torch, efm=None, n_cells=256, reps=2):
    """Precision sweep on the non-separable kernel: 3D variable hard spheres
    (gamma = 0.5), N = 64^3, M = 64 directions x 8 radial nodes (513
    transforms per evaluation), n_cells two-Gaussian mixtures (means
    U[-2,2]^3, temperatures U[0.5,1.5], seed 4001 + cell).  FP64, FP32 and
    split-BF16 evaluations timed; FP32 and split-BF16 errors against the FP64
    GPU result on every cell, and all three paths against the oracle on the
    full grid of two cells whose spectrum the oracle can afford at this plan
    (sweep_oracle_check)."""
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
    if efm is not None:
        log("bench: sweep plan vs the oracle (full grid, sparse-spectrum cells)")
        out["oracle_check"] = sweep_oracle_check(E, torch, plan, Nn, Mm, nr, gam, efm)
    out["flops_per_eval"] = flops_8d(Nn, D, plan.terms())
    for name in ("fp64", "fp32"):
        out[name]["frac_of_peak"] = round(out["flops_per_eval"] * out[name]["evals_per_s"] / 1e12
                                          / (PEAK_FP64 if name == "fp64" else PEAK_FP32), 4)
    q64 = Qs["fp64"]
    for name in ("fp32", "bf16x3"):
        d = (Qs[name] - q64).view(n_cells, -1).norm(dim=1) / q64.view(n_cells, -1).norm(dim=1)
        d = d.cpu().numpy()
        pe = np.abs(P[name] - P["fp64"]) / np.abs(P["fp64"])
        out[name].update({"rel_l2_vs_fp64_median": float(np.median(d)), "rel_l2_vs_fp64_max": float(d.max()),
                          "entropy_prod_rel_err_max": float(pe.max())})
    return out


def cpu_baseline(cells, efm, oplan, ids):
    """The oracle (plain double sum over modes of eq. Qsk, OpenMP over all
    host threads) on the full grid of the cells `ids` of the workload (the
    boundaries of the GPU passes and workgroup rounds): evals/s = cells /
    time.  Their results are also the full-grid references of the parity
    leg.  Beside it, the same fast algorithm the library runs (one forward
    and M'+1 packed inverse FFTs per cell, on the oracle's tables, torch FP64
    FFTs on the host threads): a like-for-like CPU rate for the
    transform-based method."""
    import numpy as np
    import torch
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    efm._load()
    t0 = time.perf_counter()
    refs = {c: efm.collide_modes(oplan, cells[c]) for c in ids}
    t = time.perf_counter() - t0
    out = {"value": len(ids) / t, "unit": "evals/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(ids)} of the {len(cells)} cells (ids {ids}), full 32^3 direct double "
                     f"sum over modes (M=32), {t:.1f} s"}
    # fast algorithm on the host
    torch.set_num_threads(threads)
    shp = (N,) * D
    lr, sig = oplan.lr, oplan.sigma
    G = torch.from_numpy(((lr.c[:, None] * sig * lr.U) + 1j * (sig * lr.V)).reshape((-1,) + shp))
    Dg = torch.from_numpy((sig * sig * lr.diagonal()).reshape(shp)).to(torch.complex128)
    t0 = time.perf_counter()
    k = 0
    err = None
    while k < len(ids) and (k == 0 or time.perf_counter() - t0 < 5.0):
        c = ids[k]
        F = torch.from_numpy(cells[c])
        Fh = torch.fft.fftn(F.to(torch.complex128))
        qp = torch.zeros(shp, dtype=torch.float64)
        for jj in range(G.shape[0]):
            cz = torch.fft.ifftn(G[jj] * Fh)
            qp += cz.real * cz.imag
        q = qp - F * torch.fft.ifftn(Dg * Fh).real
        if k == 0:
            err = float(np.linalg.norm(q.numpy() - refs[c].Q) / np.linalg.norm(refs[c].Qplus))
        k += 1
    t = time.perf_counter() - t0
    out["fast_fft_cpu"] = {"value": k / t, "unit": "evals/s", "cores": threads,
                           "sample": f"{k} cells, torch FP64 FFTs, {t:.1f} s",
                           "rel_l2_vs_oracle": err}
    return out, refs


def full_grid_parity(E, batches, refs, d=D, n_side=N):
    """||Q - Q_oracle||_2 / ||Q+_oracle||_2 per reference cell and path, with
    the stated bound of the path (paper_1704_07369_amd.bounds)."""
    import numpy as np
    from paper_1704_07369_amd import bounds
    out = {}
    for name, (prec, b, Q) in batches.items():
        if b is None:
            continue
        qh = E.unpack(b, Q.cpu().numpy())
        errs, bnds = [], []
        for c, ref in refs.items():
            den = np.linalg.norm(ref.Qplus)
            errs.append(float(np.linalg.norm(qh[c] - ref.Q) / den))
            bnds.append(bounds.bound(prec, n_side, d, float(np.linalg.norm(ref.Qminus) / den)))
        out[name] = {"max": max(errs), "median": float(np.median(errs)), "bound": min(bnds),
                     "within_bound": all(e <= bb for e, bb in zip(errs, bnds))}
    return out


def sweep_oracle_check(E, torch, plan, n_side, terms_m, nr, gam, efm, ncheck=2):
    """The sweep plan against the oracle on the full grid: cells that are
    real trigonometric polynomials (spectrum on 25 known modes), so the
    oracle's tables are needed on those modes only."""
    import numpy as np
    import synth
    from paper_1704_07369_amd import bounds
    inputs = [synth.trig_polynomial(7001 + c, n_side, D, L) for c in range(ncheck)]
    cells = [F for F, _ in inputs]
    refs = []
    for F, modes in inputs:
        op = efm.make_plan(n_side, D, L, terms_m, kind=efm.KIND_VHS, R=R, gamma=gam,
                           n_radial=nr, modes=modes)
        n = F.size
        q = np.empty(n); qp = np.empty(n); qm = np.empty(n)
        for i in range(0, n, 16384):
            idx = np.arange(i, min(n, i + 16384))
            q[idx], qp[idx], qm[idx], _ = efm.collide_points(op, F, idx)
        refs.append((q, qp, qm))
    out = {"cells": f"{ncheck} trigonometric polynomials (12 waves, background 1), full grid"}
    for prec, name in ((E.EC_FP64, "fp64"), (E.EC_FP32, "fp32"), (E.EC_BF16X3, "bf16x3")):
        b = E.Batch([plan], [ncheck], prec)
        f = torch.from_numpy(E.pack(b, cells)).to("cuda:0")
        Q = torch.zeros_like(f)
        b.collide(f, Q)
        qh = E.unpack(b, Q.cpu().numpy())
        errs, bnds = [], []
        for c, (q, qp, qm) in enumerate(refs):
            den = np.linalg.norm(qp)
            errs.append(float(np.linalg.norm(qh[c].ravel() - q) / den))
            bnds.append(bounds.bound(prec, n_side, D, float(np.linalg.norm(qm) / den)))
        out[name] = {"rel_l2_vs_oracle_max": max(errs), "bound": min(bnds),
                     "within_bound": all(e <= bb for e, bb in zip(errs, bnds))}
        b.close()
    return out


def c1_leg(E, torch, efm, reps):
    """The 2D configuration: N = 32^2, M = 16 (2M directions on [0, pi)),
    Maxwell molecules, L = 8, R = 6, FP64, one cell: latency per evaluation,
    and the full-grid error of the BKW datum at t = 0 and of a two-Gaussian
    mixture (seed 1001) against the oracle's double sum."""
    import numpy as np
    import synth
    from paper_1704_07369_amd import bounds
    n2, m2 = 32, 16
    p2 = E.Plan(n2, 2, L, m2, R=R)
    inputs = {"bkw": synth.bkw_datum(2, n2, L),
              "mixture": synth.sample_mixture(synth.mixture_two_gaussians(1001, 2), n2, L)}
    b, f, Q, t, _ = time_collide(E, torch, p2, [inputs["mixture"]], E.EC_FP64, reps, 2, False)
    out = {"workload": "2D Maxwell, N=32^2, M=16, L=8, R=6, FP64, one cell",
           "latency_us": t / reps * 1e6, "flops_per_eval": flops_8d(n2, 2, p2.terms())}
    b.close()
    if efm is not None:
        op = efm.make_plan(n2, 2, L, m2, R=R)
        bb = E.Batch([p2], [2], E.EC_FP64)
        ff = torch.from_numpy(E.pack(bb, list(inputs.values()))).to("cuda:0")
        QQ = torch.zeros_like(ff)
        bb.collide(ff, QQ)
        qh = E.unpack(bb, QQ.cpu().numpy())
        for k, (name, F) in enumerate(inputs.items()):
            ref = efm.collide_modes(op, F)
            out[f"{name}_rel_l2_vs_oracle"] = float(np.linalg.norm(qh[k] - ref.Q)
                                                    / np.linalg.norm(ref.Qplus))
        out["bound"] = bounds.FP64_BOUND
        bb.close()
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
    ap.add_argument("--skip-counters", action="store_true",
                    help="omit the byte-counter runs under rocprofv3 (roofline.traffic = null)")
    ap.add_argument("--counter-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--surrogate-seconds", type=float, default=40.0, help="surrogate training budget")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run ec_copy on a buffer of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): cells are independent "
              "and would be split across GPUs by cost with no exchange per step, but that "
              "split is not implemented or measured here.", file=sys.stderr)
        sys.exit(2)
    if args.counter_child:
        counter_child(args)
        return

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
    flops_eval = flops_8d(N, D, terms)

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
    efm = None
    if not args.skip_parity or not args.skip_cpu:
        from oracle import efm
    t1_64 = t1_32 = None
    reps = max(10, args.steps)
    small_us = {}
    if not args.skip_single:
        log("bench: single-cell latency")
        one = cells[:1]
        _, _, _, t1_64, _ = time_collide(E, torch, plan, one, E.EC_FP64, reps, 2, False)
        _, _, _, t1_32, _ = time_collide(E, torch, plan, one, E.EC_FP32, reps, 2, False)
        import synth
        for Ns in (16, 24):       # one cell of the smaller grids of the mixed-N leg
            ps = E.Plan(Ns, D, L, M, R=R)
            one_s = [synth.sample_mixture(synth.mixture_anisotropic(2001, D), Ns, L)]
            bs, _, _, ts, _ = time_collide(E, torch, ps, one_s, E.EC_FP64, reps, 2, False)
            small_us[f"n{Ns}_fp64_us"] = ts / reps * 1e6
            bs.close()

    traffic, traffic_note = {}, "not measured (--skip-counters)"
    if not args.skip_counters:
        log("bench: HBM byte counters (rocprofv3 --pmc child runs)")
        tr, err = measure_traffic(args)
        traffic = tr or {}
        traffic_note = err or "rocprofv3 --pmc FETCH_SIZE, WRITE_SIZE of a child run of the same batches"

    def tr_bytes(key):
        v = traffic.get(key)
        return v["bytes"] if v else None

    out = {
        "metric": METRIC, "value": ev64, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t64 / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D hard-sphere EFM collision operator, N=32^3, M=32 directions, "
                               f"L=8, R=6, batch of {args.cells} Gaussian-mixture cells, FP64",
                   "d": D, "N": N, "M": M, "L": L, "R": R, "cells": args.cells,
                   "kernel": "hard_sphere", "flops_per_eval": flops_eval},
        "roofline": roofline(prof64, flops, PEAK_FP64, tr_bytes("k_fused/f64")),
    }
    # the whole step (forward transforms included) against the same peak
    out["roofline"]["step_frac"] = round(flops_eval * args.cells / (t64 / args.steps) / 1e12
                                         / PEAK_FP64, 4)
    out["roofline"]["traffic_source"] = traffic_note
    if traffic.get("calibration"):
        out["roofline"]["traffic_calibration"] = traffic["calibration"]
    if ev32 is not None:
        r32 = roofline(prof32, flops, PEAK_FP32, tr_bytes("k_fused/f32"))
        r32["step_frac"] = round(flops_eval * args.cells / (t32 / args.steps) / 1e12 / PEAK_FP32, 4)
        out["fp32"] = {"value": ev32, "ms_per_step": t32 / args.steps * 1e3, "roofline": r32}
    if evb is not None:
        gemm = [0.0] * len(KNAMES)
        gemm[KNAMES.index("k_pencil")] = bf16_gemm_flops(N, D, terms)
        rb = roofline(profb, gemm, PEAK_BF16_MFMA, tr_bytes("k_pencil/bf16x3"), bound="mfma")
        rb["flops_note"] = ("matrix-core flops of the split-BF16 x pass: 3 products x 2 x (2N)^2 "
                            "per pencil and transform")
        out["bf16x3"] = {"value": evb, "ms_per_step": tb / args.steps * 1e3, "roofline": rb}
    if t1_64 is not None:
        out["single_cell"] = {"fp64_us": t1_64 / reps * 1e6, "fp32_us": t1_32 / reps * 1e6,
                              **small_us}
        log("bench: 2D 32^2 M=16 single cell")
        out["single_cell"]["c1_2d"] = c1_leg(E, torch, efm, reps)
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
        log("bench: mixed-N relaxation leg (200 FE steps in one captured graph)")
        out["relaxation"] = relaxation_leg(E, torch)
    if not args.skip_sweep:
        log("bench: 64^3 VHS precision sweep")
        out["precision_sweep"] = precision_sweep_leg(E, torch, efm)
    if not args.skip_surrogate:
        log("bench: learned surrogate (data, training, screened inference)")
        out["surrogate"] = surrogate_leg(E, torch, seconds=args.surrogate_seconds, log_fn=log)
        log(f"bench: surrogate {out['surrogate']}")
    if efm is not None:
        log("bench: oracle tables (quadrature)")
        oplan = efm.make_plan(N, D, L, M, R=R)
        ids = [c for c in FULL_GRID_CELLS if c < args.cells]
        log(f"bench: oracle on the full grid of cells {ids} (CPU baseline and parity)")
        base, refs = cpu_baseline(cells, efm, oplan, ids)
        if not args.skip_cpu:
            out["cpu_baseline"] = base
        if not args.skip_parity:
            out["parity"] = {
                "metric": "||Q - Q_oracle||_2 / ||Q+_oracle||_2 on the full grid of the cells "
                          f"{ids} (oracle: double sum over modes), bound stated a priori",
                **full_grid_parity(E, {"fp64": (0, b64, Q64), "fp32": (1, b32, Q32),
                                       "bf16x3": (2, bb, Qb)}, refs),
            }
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

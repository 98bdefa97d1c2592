"""Host-side logic of bench.py (no GPU): the algorithmic flop count of the
measurement rows against the values the scope table states for it, the split
of that count over the kernels, the matrix-core flops of the split-BF16 x
pass, the roofline arithmetic, the parsing of rocprofv3 counter files, and
the refusal of more than one GPU, and the end of what a counter run leaves
behind."""
import csv
import math
import os
import subprocess
import sys
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_flops_per_evaluation_match_the_stated_figures():
    # 86.58 MFLOP per 32^3 evaluation with M' = 32, 12.78 GFLOP at 64^3 with
    # M' = 512 (the measurement section of the scope table)
    assert bench.flops_8d(32, 3, 32) == pytest.approx(86.58e6, rel=1e-4)
    assert bench.flops_8d(64, 3, 512) == pytest.approx(12.78e9, rel=1e-3)
    # 2D, the single-cell configuration N = 32^2 with 2M = 32 products
    assert bench.flops_8d(32, 2, 32) == pytest.approx(
        66 * 2.5 * 1024 * 10 + 32 * (4 * 32 * 17 + 3 * 1024) + 2 * 32 * 17 + 2 * 1024)


@pytest.mark.parametrize("n_side,d,terms", [(16, 3, 32), (24, 3, 32), (32, 3, 32), (64, 3, 512),
                                            (32, 2, 32)])
def test_kernel_split_covers_the_evaluation(n_side, d, terms):
    total = bench.flops_8d(n_side, d, terms)
    k_fwd, k_pencil, k_slab, k_pipe, reserved, k_fused = bench.kernel_flops(n_side, d, terms)
    assert k_pipe == total and reserved == 0.0
    # each schedule's kernels do the whole evaluation once: two-pass k_fwd
    # (y, z), k_pencil (forward x, multiplies, inverse x), k_slab; fused: the
    # whole forward transform (2.5 n log2 n) and the fused kernel
    assert k_fwd + k_pencil + k_slab == pytest.approx(total, rel=1e-12)
    n = n_side ** d
    assert 2.5 * n * math.log2(n) + k_fused == pytest.approx(total, rel=1e-12)
    if (n_side, d) == (32, 3):
        assert k_fused == pytest.approx(85.35e6, rel=1e-4)


def test_bf16_matrix_flops():
    # three (2N x 2N) real matrix-vector products per pencil and transform
    assert bench.bf16_gemm_flops(32, 3, 32) == 3 * 2 * 64 * 64 * 32 * 32 * 33
    assert bench.bf16_gemm_flops(32, 3, 32) / 1e6 == pytest.approx(830.47, rel=1e-4)


def test_roofline_arithmetic():
    flops = bench.kernel_flops(32, 3, 32)
    ms = [2.7, 0.0, 0.0, 0.0, 0.0, 60.0]          # the fused slot dominates
    launches = [20, 0, 0, 0, 0, 20]
    prof = (ms, launches, 1024 * 20)
    r = bench.roofline(prof, flops, bench.PEAK_FP64, traffic=123)
    assert r["kernel"] == "k_fused" and r["launches"] == 20
    assert r["avg_launch_ms"] == pytest.approx(3.0)
    assert r["cells_per_launch"] == 1024
    want = flops[5] * 1024 * 20 / 60e-3 / 1e12
    assert r["achieved"] == pytest.approx(want, abs=1e-3)
    assert r["frac"] == pytest.approx(want / 78.6, abs=1e-4)
    assert r["traffic"] == 123 and r["flops_per_launch"] == pytest.approx(flops[5] * 1024)


def test_counter_files_are_summed_per_dispatch(tmp_path):
    d = tmp_path / "run" / "host"
    d.mkdir(parents=True)
    rows = [  # a counter reported in parts (per XCD) sums per dispatch
        ("1", "k_a", "10"), ("1", "k_a", "5"), ("2", "k_a", "7"), ("3", "k_b", "1.5"),
        ("3", "k_b", "0.5")]
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for disp, name, val in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": "FETCH_SIZE",
                        "Counter_Value": val})
    out = bench._read_counter_csv(str(tmp_path))
    assert sorted(out["k_a"]) == [7.0, 15.0]
    assert out["k_b"] == [2.0]


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_counter_run_leftovers_are_ended():
    # a child whose session keeps a process after the child itself exits (as
    # a profiler's helper can): the reap after the wait leaves none running
    p = subprocess.Popen(["sh", "-c", "sleep 60 & echo $!"], stdout=subprocess.PIPE, text=True,
                         start_new_session=True)
    left = int(p.stdout.readline())
    p.wait()
    os.kill(left, 0)                        # still there after the child ended
    bench._reap_group(p.pid, "test")
    deadline = time.time() + 5
    while True:
        try:
            with open(f"/proc/{left}/stat") as fh:
                if fh.read().rsplit(")", 1)[1].split()[0] == "Z":
                    break                   # ended, not yet reaped by init
        except FileNotFoundError:
            break                           # ended and reaped
        assert time.time() < deadline, "the leftover process still runs"
        time.sleep(0.01)
    bench._reap_group(p.pid, "test")        # nothing left: a no-op

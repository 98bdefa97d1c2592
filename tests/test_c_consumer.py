"""The C ABI from a plain C program (tests/c_consumer/collide_from_c.c): it
compiles as C11 against include/ec.h and links against libefm.so (CPU), and
on the GPU it builds a plan and a batch, evaluates Q and checks it (exact
zeros for F = 0, discrete mass conservation of a Gaussian cell)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_consumer", "collide_from_c.c")
LIBDIR = os.path.join(ROOT, "paper_1704_07369_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libefm.so")):
        pytest.skip("libefm.so is not built")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "collide_from_c")
    cmd = [cc, "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
           "-o", exe, "-L", LIBDIR, "-lefm", "-Wl,-rpath," + LIBDIR,
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-lm"]
    p = subprocess.run(cmd, capture_output=True, text=True)
    assert p.returncode == 0, p.stdout + p.stderr
    return exe


def test_c_consumer_compiles_and_links(tmp_path):
    _build(tmp_path)


@pytest.mark.gpu
def test_c_consumer_runs(tmp_path):
    exe = _build(tmp_path)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(p.stdout, p.stderr)
    assert p.returncode == 0 and p.stdout.strip().endswith("ok"), p.stdout + p.stderr

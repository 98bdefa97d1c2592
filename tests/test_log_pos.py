"""The logarithm of the per-cell reductions (csrc/logpos.h: frexp range
reduction to [1/sqrt 2, sqrt 2), the atanh series to s^20/21, ln 2 in two
parts), built for the host with g++ and compared with the 64-bit-mantissa
long-double logarithm: within 2 units in the last place over random
magnitudes from 1e-300 to 1e300, subnormals, values next to 1, the boundaries
of the range reduction and every power of two; log 1 = 0 exactly."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_math", "log_pos_check.cpp")
INC = os.path.join(ROOT, "paper_1704_07369_amd", "csrc")


def _values():
    rng = np.random.default_rng(7)
    v = [10.0 ** rng.uniform(-300, 300, 20000), rng.uniform(1e-20, 2.0, 5000)]
    v.append(np.array([5e-324, 1e-320, 1e-310, 2.2250738585072014e-308,
                       np.nextafter(2.2250738585072014e-308, 0.0), 1.7976931348623157e308]))
    one = np.array([1.0])
    steps = np.arange(1, 200)
    v.append(1.0 + steps * np.finfo(float).eps)
    v.append(1.0 - steps * np.finfo(float).eps / 2)
    v.append(1.0 + 10.0 ** -np.arange(1, 16, dtype=float))
    v.append(1.0 - 10.0 ** -np.arange(1, 16, dtype=float))
    for b in (0.7071067811865476, 1.4142135623730951):
        x = np.array([b])
        for _ in range(5):
            v.append(x.copy())
            x = np.nextafter(x, 2.0)
        x = np.array([b])
        for _ in range(5):
            x = np.nextafter(x, 0.0)
            v.append(x.copy())
    start = sum(len(a) for a in v)
    v.append(np.ldexp(1.0, np.arange(-1074, 1024)))
    v.append(one)
    return np.concatenate(v), start


def test_log_pos_within_two_ulp(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    exe = str(tmp_path / "log_pos_check")
    p = subprocess.run([cxx, "-std=c++17", "-O2", "-Wall", "-Werror", "-I", INC, SRC, "-o", exe],
                       capture_output=True, text=True)
    assert p.returncode == 0, p.stdout + p.stderr
    x, p2 = _values()
    out = subprocess.run([exe], input="\n".join(float(a).hex() for a in x), capture_output=True,
                         text=True, check=True).stdout.split()
    got = np.array([float.fromhex(s) for s in out])
    assert got.shape == x.shape
    ref = np.log(x.astype(np.longdouble))
    ulp = np.spacing(np.abs(ref.astype(float)))
    err = np.abs((got.astype(np.longdouble) - ref) / ulp.astype(np.longdouble)).astype(float)
    worst = int(np.argmax(err))
    print(f"largest error {err.max():.3f} ulp at x = {x[worst]!r} over {x.size} values")
    assert err.max() <= 2.0, f"{err.max():.2f} ulp at x = {x[worst]!r}"
    assert np.all(got[x == 1.0] == 0.0)
    # the powers of two: e ln 2 with ln 2 in two parts, within one ulp
    k = np.arange(-1074, 1024)
    pw = got[p2:p2 + k.size]
    assert np.all(np.abs(pw - np.log(np.ldexp(1.0, k).astype(np.longdouble)).astype(float))
                  <= np.spacing(np.abs(pw)))

"""Plan tables filled on the device against the host fill of the same tables
(ec_plan_tables against ec_host_tables).  Both evaluate the same per-mode
closed forms (sinc, the disk integral with J_1, the Chebyshev fits of the
radial factors) and the loss diagonal D (a sum of M n_radial products); they
differ only in the rounding of the device and host libm, so every entry must
agree to 1e-13 of the largest magnitude of its table row.  The host tables are
pinned to the oracle by the CPU tests."""
import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

E = pytest.importorskip("paper_1704_07369_amd")
R = 6.0


CASES = [
    # N, d, L, M, kind, gamma, n_radial, unfiltered, truncation, bcos
    (16, 2, 8.0, 16, "MAXWELL", 0.0, 0, False, "box", None),
    (64, 2, 8.0, 24, "MAXWELL", 0.0, 0, True, "box", None),
    (16, 3, 8.0, 16, "HARD_SPHERE", 1.0, 0, False, "box", None),
    (24, 3, 8.0, 12, "HARD_SPHERE", 1.0, 0, True, "box", None),
    (32, 3, 8.0, 8, "HARD_SPHERE", 1.0, 0, False, "box", None),
    (16, 3, 8.0, 8, "VHS", 0.5, 4, False, "box", None),
    (16, 3, 8.0, 8, "MAXWELL", 0.0, 4, False, "ball", None),
    (16, 3, 8.0, 8, "MAXWELL", 0.0, 3, False, "ball", [1.0, 0.5, 0.25]),
    (16, 3, 8.0, 8, "VHS", 0.5, 3, False, "box", [1.0, -0.3]),
    (64, 3, 8.0, 4, "MAXWELL", 0.0, 2, False, "ball", None),
    (128, 3, 8.0, 2, "MAXWELL", 0.0, 2, False, "ball", None),
]


@pytest.mark.parametrize("N,d,L,M,kind,gamma,nr,unf,trunc,bcos", CASES)
def test_device_tables_match_host_fill(N, d, L, M, kind, gamma, nr, unf, trunc, bcos):
    say(f"case plan tables N={N} d={d} M={M} kind={kind} gamma={gamma} n_radial={nr} "
        f"unfiltered={unf} truncation={trunc} bcos={bcos}")
    k = getattr(E, f"EC_KERNEL_{kind}")
    p = E.Plan(N, d, L, M, kind=k, R=R, gamma=gamma, n_radial=nr, filtered=not unf,
               truncation=trunc, bcos=bcos)
    dev = p.tables()
    host = E.ec_host_tables(N, d, L, p.kernel, M)
    assert dev.shape == host.shape
    scale = np.abs(host).max(axis=1, keepdims=True)
    assert np.all(scale > 0)
    err = (np.abs(dev - host) / scale).max()
    say(f"  {host.shape[0]} table rows x {host.shape[1]} modes: max rel err {err:.3e}")
    assert err <= 1e-13
    p.close()

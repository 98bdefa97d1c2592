"""Helpers for the GPU tests: run the HIP library on host arrays and bring the
results back.  torch is used only as the device allocator."""
import sys

import numpy as np


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible")
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def run_collide(E, plans, counts, cells, precision=0, chunks=None):
    """Q for every cell (list of numpy arrays), via ec_collide."""
    import torch
    b = E.Batch(plans, counts, precision)
    try:
        if chunks:
            for g, c in chunks.items():
                b.set_chunk(g, c)
        f = to_dev(E.pack(b, cells))
        Q = torch.full_like(f, float("nan"))
        b.collide(f, Q)
        torch.cuda.synchronize()
        return E.unpack(b, Q.cpu().numpy()), b
    finally:
        pass


def rel_err(q, ref, scale_ref):
    return float(np.linalg.norm((q - ref).ravel()) / np.linalg.norm(scale_ref.ravel()))


def bound_full(prec, N, d, ref):
    """Stated bound of a path (paper_1704_07369_amd.bounds) for a full-grid
    check against the oracle result ref (ratio of the loss to the gain)."""
    from paper_1704_07369_amd import bounds
    return bounds.bound(prec, N, d, float(np.linalg.norm(ref.Qminus) / np.linalg.norm(ref.Qplus)))


def bound_pts(prec, N, d, qp, qm):
    """The same bound for a check on sampled points (max-norm ratio)."""
    from paper_1704_07369_amd import bounds
    return bounds.bound(prec, N, d, float(np.abs(qm).max() / np.abs(qp).max()))

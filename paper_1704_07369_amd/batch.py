"""Owning wrappers of plan and batch handles, and host-side packing of cells
into the batch layout (marshalling only)."""
from __future__ import annotations

import numpy as np

from . import _binding as B


class Plan:
    def __init__(self, N, d, L, M, kind=None, R=6.0, gamma=None, n_radial=0, filtered=True,
                 truncation="box", bcos=None):
        """truncation "box" (|y|, |z| <= R) or "ball" (|g| <= R, the classical
        form; 3D Maxwell / VHS); bcos: coefficients of an angular factor
        b(cos theta) = sum_i bcos[i] cos^i theta (3D Maxwell / VHS)."""
        if kind is None:
            kind = B.EC_KERNEL_MAXWELL if d == 2 else B.EC_KERNEL_HARD_SPHERE
        if gamma is None:
            gamma = 0.0 if kind == B.EC_KERNEL_MAXWELL else 1.0
        if truncation not in ("box", "ball"):
            raise ValueError(f"truncation {truncation!r}: 'box' or 'ball'")
        self.N, self.d, self.L, self.M, self.kind, self.R = N, d, L, M, kind, R
        self.kernel = B.make_kernel(kind, gamma, R, n_radial, unfiltered=not filtered,
                                    truncation=B.EC_TRUNC_BALL if truncation == "ball"
                                    else B.EC_TRUNC_BOX, bcos=bcos)
        self.handle = B.ec_setup_kernel(N, d, L, self.kernel, M)

    @property
    def n(self):
        return self.N ** self.d

    @property
    def shape(self):
        return (self.N,) * self.d

    def terms(self):
        return B.ec_plan_terms(self.handle)

    def tables(self):
        return B.ec_plan_tables(self.handle, self.n)

    def close(self):
        if self.handle:
            B.ec_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    def __init__(self, plans, counts, precision=B.EC_FP64):
        self.plans = list(plans)
        self.counts = [int(c) for c in counts]
        self.precision = precision
        self.handle = B.ec_batch_create([p.handle for p in self.plans], self.counts, precision)
        self.n_cells, self.n_elems = B.ec_batch_size(self.handle)
        self.offsets = B.ec_batch_offsets(self.handle)
        self.cell_plan = []
        for p, c in zip(self.plans, self.counts):
            self.cell_plan += [p] * c

    def set_chunk(self, group, cells):
        B.ec_batch_set_chunk(self.handle, group, cells)

    def set_schedule(self, group, mode, cells=0, term_groups=0):
        B.ec_batch_set_schedule(self.handle, group, mode, cells, term_groups)

    def autotune(self, f, Q, cache_path=None, remeasure=False, stream=None):
        B.ec_autotune(self.handle, f, Q, cache_path, B.EC_TUNE_REMEASURE if remeasure else 0,
                      stream)

    def get_schedule(self, group):
        return B.ec_batch_get_schedule(self.handle, group)

    def collide(self, f, Q, stream=None):
        B.ec_collide(self.handle, f, Q, stream)

    def entropy_prod(self, f, Q, out, n_nonpos=None, stream=None):
        B.ec_entropy_prod(self.handle, f, Q, out, n_nonpos, stream)

    def monitors(self, f, Q, out, stream=None):
        B.ec_monitors(self.handle, f, Q, out, stream)

    def step(self, f, dt, n_steps, monitors=None, stream=None, method="euler"):
        """n_steps time steps in place on f: method "euler" (ec_step_graph) or
        "ssprk3" (ec_step_ssprk3)."""
        if method == "euler":
            B.ec_step_graph(self.handle, f, dt, n_steps, monitors, stream)
        elif method == "ssprk3":
            B.ec_step_ssprk3(self.handle, f, dt, n_steps, monitors, stream)
        else:
            raise ValueError(f"unknown method {method!r}")

    def profile(self, enable=True):
        B.ec_profile(self.handle, enable)

    def profile_read(self):
        return B.ec_profile_read(self.handle, len(self.plans))

    def close(self):
        if self.handle:
            B.ec_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack(batch: Batch, cells) -> np.ndarray:
    """Host array of batch.n_elems FP64 holding every cell at its offset."""
    out = np.zeros(batch.n_elems, dtype=np.float64)
    for c, arr in enumerate(cells):
        a = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        out[batch.offsets[c]: batch.offsets[c] + a.size] = a
    return out


def unpack(batch: Batch, flat) -> list:
    flat = np.asarray(flat)
    res = []
    for c, p in enumerate(batch.cell_plan):
        res.append(flat[batch.offsets[c]: batch.offsets[c] + p.n].reshape(p.shape))
    return res

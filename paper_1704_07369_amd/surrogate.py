"""Learned surrogate of the collision operator: owning wrapper, training data
from the exact operator's own relaxation trajectories, training loop and
screened inference (marshalling and orchestration; every computation runs in
libefm.so)."""
from __future__ import annotations

import time

import numpy as np

from . import _binding as B
from .batch import Batch, Plan, pack

# network of the learned surrogate: 4 layers, 16 channels, 12 modes per axis
DEFAULT = dict(modes=12, channels=16, layers=4)

# Stated accuracy of the screened surrogate: relative L2 error of every
# accepted cell's Q against the exact FP64 operator <= SURROGATE_BOUND; cells
# failing the screen take the exact operator's Q.  Default screen: discrete
# H-functional of the projected Q <= 0 (Theorem 1) and mass residual of the
# raw prediction <= 5e-3; no momentum/energy check (tau_e < 0).
SURROGATE_BOUND = 5e-2
SCREEN_TAU_M = 5e-3
SCREEN_TAU_E = -1.0


class Surrogate:
    def __init__(self, N=32, modes=12, channels=16, layers=4, seed=1234, max_batch=16):
        self.N, self.modes, self.channels, self.layers = N, modes, channels, layers
        self.max_batch = max_batch
        self.handle = B.ec_surrogate_create(N, modes, channels, layers, seed, max_batch)

    @property
    def n_params(self):
        return B.ec_surrogate_num_params(self.handle)

    def params(self):
        return B.ec_surrogate_get_params(self.handle)

    def set_params(self, p):
        B.ec_surrogate_set_params(self.handle, p)

    def grads(self):
        return B.ec_surrogate_get_grads(self.handle)

    def prepare(self, batch: Batch, f, Q, cell0, nb, Fin, target):
        B.ec_surrogate_prepare(self.handle, batch.handle, f, Q, cell0, nb, Fin, target)

    def forward(self, Fin, y, nb):
        B.ec_surrogate_forward(self.handle, Fin, y, nb)

    def train_step(self, Fin, target, nb, lr, update=True, want_loss=True):
        return B.ec_surrogate_train(self.handle, Fin, target, nb, lr, update, want_loss)

    def collide(self, batch: Batch, f, Q, tau_m=SCREEN_TAU_M, tau_e=SCREEN_TAU_E, fell_back=None,
                screen=None):
        return B.ec_surrogate_collide(self.handle, batch.handle, f, Q, tau_m, tau_e, fell_back,
                                      screen)

    def close(self):
        if self.handle:
            B.ec_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def generate_pairs(torch, plan: Plan, cells, n_steps, dt, sur: Surrogate):
    """(c0 F/mass, c0^2 Q/mass^2) pairs along forward-Euler trajectories of the exact
    operator (ec_collide + ec_step), stored on the device as FP32 tensors of
    shape [len(cells) * n_steps, N^3]."""
    nc = len(cells)
    b = Batch([plan], [nc])
    f = torch.from_numpy(pack(b, cells)).to("cuda:0")
    Q = torch.zeros_like(f)
    n = plan.n
    Fin = torch.empty((nc * n_steps, n), dtype=torch.float32, device="cuda:0")
    Tgt = torch.empty_like(Fin)
    mb = sur.max_batch
    for s in range(n_steps):
        b.collide(f, Q)
        for c0 in range(0, nc, mb):
            k = min(mb, nc - c0)
            row = s * nc + c0
            sur.prepare(b, f, Q, c0, k, Fin[row:row + k], Tgt[row:row + k])
        b.step(f, dt, 1)
    torch.cuda.synchronize()
    return Fin, Tgt


def train(torch, sur: Surrogate, Fin, Tgt, seconds=60.0, batch=16, lr=1e-3, seed=0, log=None):
    """Adam on random minibatches until the time budget is spent; returns the
    loss history (mean relative squared error per logged step)."""
    rng = np.random.default_rng(seed)
    npairs = Fin.shape[0]
    xb = torch.empty((batch, Fin.shape[1]), dtype=torch.float32, device="cuda:0")
    tb = torch.empty_like(xb)
    hist = []
    t0 = time.perf_counter()
    step = 0
    while time.perf_counter() - t0 < seconds:
        idx = torch.from_numpy(rng.choice(npairs, batch, replace=False)).to("cuda:0")
        torch.index_select(Fin, 0, idx, out=xb)
        torch.index_select(Tgt, 0, idx, out=tb)
        frac = min(1.0, (time.perf_counter() - t0) / seconds)
        cur_lr = lr * 0.5 * (1.0 + np.cos(np.pi * frac))     # cosine decay
        want = step % 50 == 0
        loss = sur.train_step(xb, tb, batch, cur_lr, True, want)
        if want:
            hist.append((step, time.perf_counter() - t0, loss))
            if log:
                log(f"surrogate step {step}: loss {loss:.4e}")
        step += 1
    torch.cuda.synchronize()
    return hist, step

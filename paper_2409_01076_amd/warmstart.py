"""Learned warm starts for the lid-driven cavity.

A coordinate network (``smrt.MLP``: bf16 matrix-core kernels, FP32
accumulation) maps a node centre (x, y) in [0, 1]^2 and the Reynolds number to
(rho, u, v) of the steady flow.  It is trained on steady fields that the cavity
solver itself produced, and its prediction sets the initial populations
f = f^eq(rho, u) of a new run instead of the uniform cold start; the lattice
Boltzmann run to the same residual then removes whatever error the prediction
has, so the final field is the solver's, not the network's.

Inputs: s = log(Re / 100) / log(100), so Re in [100, 10^4] maps to [0, 1].
Targets: ((rho - 1) * RHO_SCALE, u / U, v / U).  The predicted density is
rescaled so the total mass equals the cold start's (N^2): the closed cavity
conserves mass, so the initial mass fixes the final state.

Only orchestration lives here: every arithmetic step of training and
inference runs in the library's kernels; numpy draws the shuffle order (a
device gather applies it) and does the host-side bookkeeping.
"""
import math
import time

import numpy as np
import torch

from . import smrt

RHO_SCALE = 100.0


def re_coordinate(re):
    return math.log(float(re) / 100.0) / math.log(100.0)


def cavity_points(n, re):
    """(n*n, 3) float32 array of (x, y, s), rows in [y][x] order."""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    y, x = np.meshgrid(c, c, indexing="ij")
    s = np.full(n * n, re_coordinate(re))
    return np.stack([x.ravel(), y.ravel(), s], axis=1).astype(np.float32)


def targets(rho, ux, uy, u_lid):
    return np.stack([(np.ravel(rho) - 1.0) * RHO_SCALE, np.ravel(ux) / u_lid, np.ravel(uy) / u_lid],
                    axis=1).astype(np.float32)


class WarmStart:
    """Network + fixed Fourier frequencies + training loop."""

    def __init__(self, fourier=16, width=128, layers=5, batch=65536, fourier_sigma=2.0, seed=2409,
                 device="cuda:0"):
        self.device = torch.device(device)
        self.batch = batch
        self.net = smrt.MLP(fourier=fourier, width=width, layers=layers, outputs=3,
                            max_batch=batch, device=device)
        rng = np.random.default_rng(seed)
        self.B = rng.normal(0.0, fourier_sigma, size=(fourier, 3)).astype(np.float32)
        params = []
        dims = [3 + 2 * fourier] + [width] * (layers - 1) + [3]
        for i, o in zip(dims[:-1], dims[1:]):
            bound = math.sqrt(6.0 / (i + o))
            params.append(rng.uniform(-bound, bound, size=i * o))
            params.append(np.zeros(o))
        p = np.concatenate(params).astype(np.float32)
        assert p.size == self.net.param_count
        self.net.set_params(torch.from_numpy(p).to(self.device), torch.from_numpy(self.B).to(self.device))

    def close(self):
        self.net.close()

    def fit(self, points, target, epochs=20, lr=2e-3, lr_min=2e-5, seed=7, log=None):
        """points, target: host float32 arrays (N, 3).  Mini-batches of
        `batch` rows from one shuffled order; cosine learning-rate decay.
        Returns the list of (step, loss) recorded once per epoch."""
        bs = min(self.batch, (points.shape[0] // 64) * 64)
        if bs == 0:
            raise ValueError("need at least 64 training rows")
        n = (points.shape[0] // bs) * bs
        order = torch.from_numpy(np.random.default_rng(seed).permutation(points.shape[0])[:n]).to(self.device)
        # shuffled on the device: one upload of the rows, then a gather
        P = torch.from_numpy(np.ascontiguousarray(points, dtype=np.float32)).to(self.device)[order].contiguous()
        T = torch.from_numpy(np.ascontiguousarray(target, dtype=np.float32)).to(self.device)[order].contiguous()
        per_epoch = n // bs
        total = epochs * per_epoch
        history = []
        t0 = time.perf_counter()
        for e in range(epochs):
            for b in range(per_epoch):
                step = e * per_epoch + b
                rate = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / total))
                last = b == per_epoch - 1
                loss = self.net.train_step(P[b * bs:(b + 1) * bs], T[b * bs:(b + 1) * bs], rate,
                                           want_loss=last)
            history.append((total if e == epochs - 1 else (e + 1) * per_epoch, loss))
            if log:
                log("epoch %d loss %.4e (%.1f s)" % (e + 1, loss, time.perf_counter() - t0))
        torch.cuda.synchronize(self.device)
        return history

    def predict(self, n, re, u_lid):
        """(rho, ux, uy) float32 device tensors (n, n) for a cavity of side n,
        rho rescaled to total mass n^2."""
        pts = cavity_points(n, re)
        rows = pts.shape[0]
        padded = -(-rows // 64) * 64
        out = torch.empty((padded, 3), dtype=torch.float32, device=self.device)
        P = torch.zeros((padded, 3), dtype=torch.float32, device=self.device)
        P[:rows].copy_(torch.from_numpy(pts))
        for s in range(0, padded, self.batch):
            e = min(padded, s + self.batch)
            self.net.forward(P[s:e], out[s:e])
        y = out[:rows].cpu().numpy().astype(np.float64)
        rho = 1.0 + y[:, 0] / RHO_SCALE
        rho *= rows / rho.sum()
        ux, uy = y[:, 1] * u_lid, y[:, 2] * u_lid
        to = lambda a: torch.from_numpy(a.reshape(n, n).astype(np.float32)).to(self.device)
        return to(rho), to(ux), to(uy)

"""Training the pressure warm-start network on solver snapshots.

A snapshot is what the library records at each pressure solve while a
network is attached (include/vos_unet.h): the network input [eps_s, scaled
initial residual, x position, 1] and the increment p^{n+1} - p^n the solve
produced, scaled by gain * s0.  Collection, training and evaluation all run
through the C ABI; this module only moves tensors around.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import unet as U
from . import vos


@dataclass
class Dataset:
    x: "object"      # torch (S, nz, ny, nx, 4) float32 on the device
    t: "object"      # torch (S, nz, ny, nx) float32: each increment scaled to unit rms
    gain: float      # rms of the raw targets (increment / s0) over the set


def collect(sim: vos.Sim, steps: int, dt: float, probe: U.UNet, gain_collect: float = 1.0) -> Dataset:
    """Advance `sim` `steps` steps with `probe` attached (guess off) and keep
    every step's snapshot.  The solver rescales the network output by a line
    search, so only the shape of the increment is learned: each target is
    scaled to unit rms."""
    torch = sim.torch
    U.attach(sim, probe, gain=gain_collect, use_guess=False)
    xs, ts = [], []
    for _ in range(steps):
        sim.step(dt)
        x, t = U.warm_start_sample(sim)
        xs.append(x)
        ts.append(t)
    U.attach(sim, None)
    X = torch.stack(xs)
    T = torch.stack(ts).double()
    r = torch.sqrt(torch.mean(T ** 2, dim=tuple(range(1, T.dim())), keepdim=True))
    rms = float(torch.sqrt(torch.mean(T ** 2)))
    T = torch.where(r > 0, T / torch.where(r > 0, r, torch.ones_like(r)), torch.zeros_like(T))
    return Dataset(X, T.float().contiguous(), gain_collect * (rms if rms > 0 else 1.0))


def train(net: U.UNet, data: Dataset, iters: int, lr: float = 1e-3, seed: int = 0, log_every: int = 0):
    """Adam on random mini-batches of the net's planned batch size; returns the
    loss history."""
    torch = net.torch
    b = net.shape[0]
    S = data.x.shape[0]
    g = np.random.default_rng(seed)
    hist = []
    xb = torch.empty((b,) + tuple(data.x.shape[1:]), dtype=torch.float32, device=net.device)
    tb = torch.empty((b,) + tuple(data.t.shape[1:]), dtype=torch.float32, device=net.device)
    for it in range(iters):
        idx = torch.as_tensor(g.integers(0, S, b), device=net.device)
        torch.index_select(data.x, 0, idx, out=xb)
        torch.index_select(data.t, 0, idx, out=tb)
        torch.cuda.current_stream(net.device).synchronize()
        want = log_every and (it % log_every == 0 or it == iters - 1)
        loss = net.train_step(xb, tb, lr, want_loss=bool(want) or it == iters - 1)
        if loss is not None:
            hist.append((it, loss))
    net.stream.synchronize()
    return hist

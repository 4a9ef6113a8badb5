"""FP64 NumPy oracle of the pressure warm-start U-Net -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this module.  The product library never calls it and shares no
code with it.

The network is not in the paper (its outlook names learned models as future
work); it is the learned initial guess of the pressure-correction solve.  What
it computes has a plain definition, written out here:

  3 levels with 16 / 32 / 64 channels, every convolution 3x3x3 with zero
  padding, bias and ReLU; 2x2x2 average pooling down, nearest-neighbour 2x
  upsampling up, skip connections by channel concatenation [upsampled, skip];
  a 1x1x1 head 16 -> 1 without activation; loss = mean squared error.

  level 0:  X0 (cin padded to 16) -e0a-> A0 (16) -e0b-> S0 (16)
  level 1:  pool S0 -e1a-> A1 (32) -e1b-> S1 (32)
  level 2:  pool S1 -ba-> A2 (64) -bb-> B2 (64)
  level 1:  [up B2, S1] (96) -d1a-> (32) -d1b-> E1 (32)
  level 0:  [up E1, S0] (48) -d0a-> (16) -d0b-> E0 (16) -head-> y

Activations are NDHWC (x fastest among D, H, W), weights W[tap][ci][co] with
tap = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), and the tap reads x[z+dz, y+dy, x+dx].

``bf16=True`` rounds to bfloat16 (round to nearest even) at the points where
the mixed-precision network stores bfloat16: the packed input, the conv
weights, every stored activation and every stored activation gradient.  The
arithmetic between those points stays FP64.  ``bf16=False`` is the plain FP64
network (used by the finite-difference pins).

The backward pass is the adjoint of each forward operation, written out; Adam
follows Kingma & Ba (2015), Algorithm 1, with bias correction.
"""
from __future__ import annotations

import numpy as np

LAYERS = (  # name, input channels, output channels
    ("e0a", 16, 16), ("e0b", 16, 16),
    ("e1a", 16, 32), ("e1b", 32, 32),
    ("ba", 32, 64), ("bb", 64, 64),
    ("d1a", 96, 32), ("d1b", 32, 32),
    ("d0a", 48, 16), ("d0b", 16, 16),
)


def n_params() -> int:
    return sum(27 * ci * co + co for _, ci, co in LAYERS) + 17


def unpack(theta: np.ndarray) -> dict:
    """Flat parameter vector -> {name: (W[27, ci, co], b[co])}, 'head': (w[16], b[1])."""
    p, o = {}, 0
    for name, ci, co in LAYERS:
        w = theta[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        b = theta[o:o + co]
        o += co
        p[name] = (w, b)
    p["head"] = (theta[o:o + 16], theta[o + 16:o + 17])
    assert o + 17 == theta.size
    return p


def pack(p: dict) -> np.ndarray:
    parts = []
    for name, _, _ in LAYERS:
        parts += [p[name][0].ravel(), p[name][1].ravel()]
    parts += [p["head"][0].ravel(), p["head"][1].ravel()]
    return np.concatenate(parts)


def bf16(a):
    """Round to bfloat16 (nearest, ties to even), returned as float64.

    FP64 is first rounded to FP32 (the GPU rounds FP32 accumulators)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _taps():
    for tap in range(27):
        yield tap, tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1


def conv3d(x, w, b=None):
    """y[v] = sum over taps of x[v + off(tap)] W[tap] (+ b), zeros outside."""
    N, D, H, W_, ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((N, D, H, W_, w.shape[2]))
    for tap, dz, dy, dx in _taps():
        y += xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W_, :] @ w[tap]
    if b is not None:
        y += b
    return y


def conv3d_dgrad(g, w):
    """Adjoint of conv3d in x: dx[v + off(tap)] += g[v] W[tap]^T."""
    N, D, H, W_, _ = g.shape
    dxp = np.zeros((N, D + 2, H + 2, W_ + 2, w.shape[1]))
    for tap, dz, dy, dx in _taps():
        dxp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W_, :] += g @ w[tap].T
    return dxp[:, 1:-1, 1:-1, 1:-1, :]


def conv3d_wgrad(x, g):
    """dW[tap] = sum over voxels of x[v + off(tap)]^T g[v]."""
    N, D, H, W_, ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros((27, ci, g.shape[4]))
    gm = g.reshape(-1, g.shape[4])
    for tap, dz, dy, dx in _taps():
        xs = xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W_, :].reshape(-1, ci)
        dw[tap] = xs.T @ gm
    return dw


def pool(x):
    """2x2x2 average pooling."""
    N, D, H, W_, C = x.shape
    return x.reshape(N, D // 2, 2, H // 2, 2, W_ // 2, 2, C).mean(axis=(2, 4, 6))


def pool_adjoint(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up(x):
    """Nearest-neighbour 2x upsampling."""
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up_adjoint(g):
    N, D, H, W_, C = g.shape
    return g.reshape(N, D // 2, 2, H // 2, 2, W_ // 2, 2, C).sum(axis=(2, 4, 6))


def forward(theta, x, bf16_round: bool = True):
    """x: (N, D, H, W, cin) with cin <= 16.  Returns (y[N, D, H, W], cache)."""
    q = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(np.asarray(theta, dtype=np.float64))
    N, D, H, W_, cin = x.shape
    assert cin <= 16 and D % 4 == 0 and H % 4 == 0 and W_ % 4 == 0
    X0 = np.zeros((N, D, H, W_, 16))
    X0[..., :cin] = q(x)

    def conv(name, inp):
        w, b = p[name]
        return q(np.maximum(conv3d(inp, q(w), b), 0.0))

    c = {"X0": X0}
    c["A0"] = conv("e0a", X0)
    c["S0"] = conv("e0b", c["A0"])
    c["P0"] = q(pool(c["S0"]))
    c["A1"] = conv("e1a", c["P0"])
    c["S1"] = conv("e1b", c["A1"])
    c["P1"] = q(pool(c["S1"]))
    c["A2"] = conv("ba", c["P1"])
    c["B2"] = conv("bb", c["A2"])
    c["C1"] = np.concatenate([up(c["B2"]), c["S1"]], axis=4)
    c["D1"] = conv("d1a", c["C1"])
    c["E1"] = conv("d1b", c["D1"])
    c["C0"] = np.concatenate([up(c["E1"]), c["S0"]], axis=4)
    c["D0"] = conv("d0a", c["C0"])
    c["E0"] = conv("d0b", c["D0"])
    hw, hb = p["head"]
    y = c["E0"] @ hw + hb[0]
    return y, c


def loss_and_grad(theta, x, target, bf16_round: bool = True):
    """MSE loss mean((y - t)^2) and its gradient in the flat parameter order."""
    q = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(np.asarray(theta, dtype=np.float64))
    y, c = forward(theta, x, bf16_round)
    V = y.size
    r = y - target
    loss = float(np.sum(r * r) / V)
    dy = 2.0 * r / V
    g = {}
    hw, hb = p["head"]
    g["head"] = (np.einsum("ndhwc,ndhw->c", c["E0"], dy), np.array([dy.sum()]))

    def relu_mask(grad, act):
        return np.where(act > 0.0, grad, 0.0)

    def back(name, inp, gout, mask_with=None):
        """Gradient of a conv layer given the gradient of its pre-activation."""
        w, _ = p[name]
        g[name] = (conv3d_wgrad(inp, gout), gout.sum(axis=(0, 1, 2, 3)))
        if mask_with is None:
            return None
        return q(relu_mask(conv3d_dgrad(gout, q(w)), mask_with))

    gE0 = q(relu_mask(dy[..., None] * hw, c["E0"]))
    gD0 = back("d0b", c["D0"], gE0, c["D0"])
    gC0 = back("d0a", c["C0"], gD0, c["C0"])
    gE1 = q(up_adjoint(gC0[..., :32]))
    gD1 = back("d1b", c["D1"], gE1, c["D1"])
    gC1 = back("d1a", c["C1"], gD1, c["C1"])
    gB2 = q(up_adjoint(gC1[..., :64]))
    gA2 = back("bb", c["A2"], gB2, c["A2"])
    gP1 = q(conv3d_dgrad(gA2, q(p["ba"][0])))
    back("ba", c["P1"], gA2)
    gS1 = q(gC1[..., 64:] + relu_mask(pool_adjoint(gP1), c["S1"]))
    gA1 = back("e1b", c["A1"], gS1, c["A1"])
    gP0 = q(conv3d_dgrad(gA1, q(p["e1a"][0])))
    back("e1a", c["P0"], gA1)
    gS0 = q(gC0[..., 32:] + relu_mask(pool_adjoint(gP0), c["S0"]))
    gA0 = back("e0b", c["A0"], gS0, c["A0"])
    back("e0a", c["X0"], gA0)
    return loss, pack(g), y


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1); t counts from 1.

    Returns (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v

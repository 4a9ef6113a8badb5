"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the oracle.

This module holds geometry generators and workload parameters only -- none of
the method's arithmetic.  The paper's own geometries (the calcite post, the
micromodel image, the Ketton micro-CT; Section 3) are not available, so these
generators stand in for them with the same structure:

* ``calcite_post``   -- one binary disc in a 2-D channel (Benchmark 1 stand-in);
* ``rsa_discs``      -- non-overlapping polydisperse discs placed by random
                        sequential addition (Benchmark 2 micromodel stand-in);
* ``sphere_pack``    -- overlapping log-normal spheres with partial-volume
                        interface voxels and sub-voxel noise (Benchmark 3
                        Ketton stand-in).

Every array returned is the solid fraction eps_s in [0, 1], shaped (nz, ny, nx),
x fastest.  All randomness comes from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np

# Physical parameters shared by the workloads (SI, mol).  rho is the fluid
# density; Vm = M_ws / rho_s = 100 kg/kmol / 2710 kg/m3 (calcite, Table 1).
BASE_PARAMS = dict(mu=1e-3, rho=1000.0, D=1e-9, k0=1e-15, kc=1e-4, Vm=3.69e-5, zeta=1.0,
                   c_in=10.0, eps_min=1e-4, u_in=1e-4, p_out=0.0)


def calcite_post(nx: int = 256, ny: int = 64, cx: int = 64, cy: int = 32, r: int = 20) -> np.ndarray:
    """Binary disc: cell (i, j) is solid iff (i - cx)^2 + (j - cy)^2 <= r^2."""
    j, i = np.mgrid[0:ny, 0:nx]
    es = ((i - cx) ** 2 + (j - cy) ** 2 <= r * r).astype(np.float64)
    return es.reshape(1, ny, nx)


def rsa_discs(nx: int, ny: int, seed: int, rmin: float = 10.0, rmax: float = 40.0,
              porosity: float = 0.6, gap: float = 2.0, band: int = 2,
              max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition of non-overlapping discs.

    Radii are uniform in [rmin, rmax] cells (real-valued); a disc is accepted if
    it lies inside the domain minus a ``band``-cell margin on every side and
    keeps a gap of at least ``gap`` cells to every accepted disc.  Addition
    stops at the first porosity <= ``porosity`` (or after ``max_tries``).
    Rasterisation is binary on cell centres (i + 0.5, j + 0.5).
    """
    rng = np.random.default_rng(seed)
    solid = np.zeros((ny, nx), dtype=bool)
    discs = []
    jj, ii = np.mgrid[0:ny, 0:nx]
    xc_all = ii + 0.5
    yc_all = jj + 0.5
    for _ in range(max_tries):
        r = rng.uniform(rmin, rmax)
        lo_x, hi_x = band + r, nx - band - r
        lo_y, hi_y = band + r, ny - band - r
        if hi_x <= lo_x or hi_y <= lo_y:
            continue
        cx = rng.uniform(lo_x, hi_x)
        cy = rng.uniform(lo_y, hi_y)
        ok = True
        for (ox, oy, orr) in discs:
            if (cx - ox) ** 2 + (cy - oy) ** 2 < (r + orr + gap) ** 2:
                ok = False
                break
        if not ok:
            continue
        discs.append((cx, cy, r))
        x0, x1 = max(0, int(cx - r) - 1), min(nx, int(cx + r) + 2)
        y0, y1 = max(0, int(cy - r) - 1), min(ny, int(cy + r) + 2)
        sub = (xc_all[y0:y1, x0:x1] - cx) ** 2 + (yc_all[y0:y1, x0:x1] - cy) ** 2 <= r * r
        solid[y0:y1, x0:x1] |= sub
        if 1.0 - solid.mean() <= porosity:
            break
    return solid.astype(np.float64).reshape(1, ny, nx)


def sphere_pack(n: int, seed: int, median_r: float = 20.0, sigma: float = 0.3,
                porosity: float = 0.23, noise: float = 0.01, band: int = 2,
                ny: int | None = None, nz: int | None = None) -> np.ndarray:
    """Overlapping spheres with log-normal radii r = median_r * exp(sigma N(0,1)),
    centres uniform in the box, added until the porosity first drops to
    ``porosity``.  The solid fraction of a voxel is the partial-volume ramp
    clip(0.5 - d, 0, 1) of the signed distance d (in voxels) from its centre to
    the union surface; interface voxels (0 < eps_s < 1) get additive
    N(0, noise) and are clipped to [0, 1].  ``band`` voxel planes at the inlet
    (x = 0) and outlet (x = n - 1) are set to fluid.
    """
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    dist = np.full((nz, ny, nx), np.inf, dtype=np.float32)
    tot = nx * ny * nz

    def frac_solid() -> float:
        return float(np.clip(0.5 - dist, 0.0, 1.0).sum(dtype=np.float64)) / tot

    batch = 8
    while True:
        for _ in range(batch):
            r = median_r * float(np.exp(sigma * rng.standard_normal()))
            c = rng.uniform([0, 0, 0], [nx, ny, nz])
            lo = np.maximum(np.floor(c - r - 1).astype(int), 0)
            hi = np.minimum(np.ceil(c + r + 1).astype(int), [nx, ny, nz])
            if np.any(hi <= lo):
                continue
            zs = np.arange(lo[2], hi[2]) + 0.5
            ys = np.arange(lo[1], hi[1]) + 0.5
            xs = np.arange(lo[0], hi[0]) + 0.5
            d = np.sqrt((zs[:, None, None] - c[2]) ** 2 + (ys[None, :, None] - c[1]) ** 2
                        + (xs[None, None, :] - c[0]) ** 2) - r
            view = dist[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            np.minimum(view, d.astype(np.float32), out=view)
        if 1.0 - frac_solid() <= porosity:
            break
    es = np.clip(0.5 - dist.astype(np.float64), 0.0, 1.0)
    iface = (es > 0.0) & (es < 1.0)
    es[iface] += noise * rng.standard_normal(int(iface.sum()))
    np.clip(es, 0.0, 1.0, out=es)
    es[:, :, :band] = 0.0
    es[:, :, nx - band:] = 0.0
    return es


def workload(name: str):
    """Named workloads: geometry (eps_s) and parameter overrides.

    ``post``       256x64 2-D calcite post, dx = 5 um, 20 steps of 1 ms (iVoS, FP64).
    ``micromodel`` 1024x512 2-D RSA disc micromodel, dx = 5 um (seed 11).
    ``pack``       256^3 sphere pack, dx = 4 um (seed 33).
    """
    if name == "post":
        return calcite_post(), dict(BASE_PARAMS, dx=5e-6)
    if name == "micromodel":
        return rsa_discs(1024, 512, seed=11), dict(BASE_PARAMS, dx=5e-6)
    if name == "pack":
        return sphere_pack(256, seed=33), dict(BASE_PARAMS, dx=4e-6)
    raise KeyError(name)


# Layer shapes of the warm-start U-Net (input channels, output channels), in
# parameter order; the flat parameter vector holds, per layer, W[27][ci][co]
# then b[co], followed by the 1x1x1 head's w[16] and b[1].
UNET_LAYERS = ((16, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64),
               (96, 32), (32, 32), (48, 16), (16, 16))


def unet_init(seed: int, cin: int = 4) -> np.ndarray:
    """He-normal conv weights (fan-in 27 * real input channels), zero biases,
    small normal head; weights of padded input channels (>= cin) are zero.
    Returns the flat FP32 parameter vector."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(UNET_LAYERS):
        real = cin if li == 0 else ci
        w = rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * real))
        if li == 0:
            w[:, cin:, :] = 0.0
        parts += [w.ravel(), np.zeros(co)]
    parts += [rng.standard_normal(16) * 0.25, np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def unet_batch(n: int, d: int, h: int, w: int, seed: int, cin: int = 4):
    """Synthetic U-Net inputs (n, d, h, w, cin) in FP32 and a smooth target
    (n, d, h, w): channel 0 a solid fraction in [0, 1], the others smooth
    fields; the target is a fixed nonlinear mix of them."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.linspace(0, 1, d), np.linspace(0, 1, h), np.linspace(0, 1, w), indexing="ij")
    xs = np.zeros((n, d, h, w, cin), np.float32)
    t = np.zeros((n, d, h, w), np.float32)
    for b in range(n):
        f = rng.uniform(1.0, 3.0, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        xs[b, ..., 0] = (rng.random((d, h, w)) < 0.3).astype(np.float32)
        for c in range(1, cin):
            xs[b, ..., c] = np.sin(2 * np.pi * f[c % 3] * [x, y, z][c % 3] + ph[c % 3])
        t[b] = xs[b, ..., 1] * (1.0 - xs[b, ..., 0]) + 0.5 * x
    return xs, t

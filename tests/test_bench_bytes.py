"""The algorithmic byte count that bench.py divides by the pressure-solve time,
checked against an enumeration of the launches of one pressure CG iteration
on a 256^3 grid, array by array (host logic only)."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

N = 256
TAIL = 4096  # levels of at most this many cells run in the single-block tail


def march_levels():
    n, out = N, []
    while n ** 3 > TAIL:
        out.append(n ** 3)
        n //= 2
    return out


def vcycle_launches(nu, w):
    """(cells of the level, bytes per level cell) of every fine-level launch
    of a 3-D pressure V-cycle; FP64 residual in and result out on level 0."""
    T = 3 * w              # the three face arrays around a cell (one per cell each)
    cells = march_levels()
    out = []
    for l, nc in enumerate(cells):
        fine = l == 0
        diag = 0 if fine else w   # the finest level forms it from the faces
        out.append((nc, (8 if fine else w) + w + T + (w if fine else 0) + w))   # sweeps 1-2: r or b, diag, T -> (b), x
        for _ in range(nu - 2):
            out.append((nc, w + w + diag + T + w))                         # x, b, diag, T -> x'
        out.append((nc, w + w + diag + T + w / 8))                         # residual restricted to coarse b
    for l, nc in reversed(list(enumerate(cells))):
        fine = l == 0
        diag = 0 if fine else w
        out.append((nc, w + w / 8 + w + diag + T + w))                     # x + coarse x, b, diag, T -> x'
        for k in range(1, nu):
            last = fine and k == nu - 1
            out.append((nc, w + w + diag + T + w + (8 if last else 0)))    # (last: FP64 result z)
    return out


@pytest.mark.parametrize("tag,w", [("fp64", 8), ("mixed", 4)])
@pytest.mark.parametrize("nu", [2, 3, 4])
def test_pressure_iteration_bytes_3d(tag, w, nu):
    nc = N ** 3
    cg = nc * (8 + 3 * 8 + 8) + nc * 56 + nc * 24 + nc * 24   # apply, x/r update, z.r z.q, direction
    enum = cg + sum(c * b for c, b in vcycle_launches(nu, w))
    model = bench.p_iter_bytes(3, tag, nu) * nc
    # the model sums the coarser levels to infinity; the enumeration stops at the tail
    assert model == pytest.approx(enum, rel=2e-3)


def test_pressure_iteration_bytes_2d():
    # tiled legs: level 0 down r 8 + (diag, 2 T, b, x, coarse b/4), up (x, coarse x/4, b, diag, 2 T, result) + z 8
    for tag, w in (("fp64", 8), ("mixed", 4)):
        levels = [4 ** -l for l in range(12)]
        v = 16 + sum(f * (5.25 * w + 6.25 * w) for f in levels)
        assert bench.p_iter_bytes(2, tag) == pytest.approx(136 + v, rel=1e-5)

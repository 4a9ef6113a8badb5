"""Upscaling workload (Section 2.5; the fits of Sections 3.2 and 3.3): a long
dissolution run on the GPU step, recording the whole-domain porosity phi,
permeability K, correction factor alpha, specific surface area a and Darcy
velocity U_D, and power-law fits K = C phi^n, alpha = C phi^m -- one law, or
two laws split where the fit is best (the wormhole regime's change of slope
at reactant breakthrough, Section 3.3).

Every step runs in the library (vos_step); this module only orders the steps,
reads the diagnostics the step returns and fits them on the host.  The solid
step is bounded by the simulation's deps_max (Appendix D), so a run advances
by steps of at most that change of the fluid fraction; the flow and transport
of a step are solved on the porosity at its start, which is the phi recorded
beside that step's K and alpha.
"""
from __future__ import annotations

import time

import numpy as np


def fit_power_law(phi, y):
    """(C, n, rms) of y = C phi^n: a straight line through (log phi, log y)
    by numpy's least squares; rms is the root mean square log residual."""
    x = np.log(np.asarray(phi, dtype=np.float64))
    v = np.log(np.asarray(y, dtype=np.float64))
    if x.size < 2 or np.ptp(x) == 0.0:
        raise ValueError("need two distinct porosities")
    A = np.stack([np.ones_like(x), x], axis=1)
    (lc, n), *_ = np.linalg.lstsq(A, v, rcond=None)
    r = v - (lc + n * x)
    return float(np.exp(lc)), float(n), float(np.sqrt(np.mean(r * r)))


def fit_two_power_laws(phi, y, min_points=3):
    """(k, (C1, n1, rms1), (C2, n2, rms2)): points [0, k) follow the first law,
    [k, m) the second; k minimises the summed squared log residual of the two
    fits (each side at least min_points)."""
    m = len(phi)
    if m < 2 * min_points:
        raise ValueError("too few points for two laws")
    best = None
    for k in range(min_points, m - min_points + 1):
        f1 = fit_power_law(phi[:k], y[:k])
        f2 = fit_power_law(phi[k:], y[k:])
        ss = f1[2] ** 2 * k + f2[2] ** 2 * (m - k)
        if best is None or ss < best[0]:
            best = (ss, k, f1, f2)
    return best[1], best[2], best[3]


def run(sim, dt, max_steps, target_porosity=None, time_budget=None, volume=None):
    """Advance sim until its porosity reaches target_porosity (or max_steps,
    or time_budget seconds of wall time).  Returns per-step arrays phi, K,
    alpha, a, U_D, t (simulated time at the step's end), dt_solid, outer_its,
    and the wall time."""
    eps = sim.get("eps")
    phi = float(eps.mean().item())
    if volume is None:
        volume = float(eps.numel()) * sim.grid.dx ** 3
    del eps
    rec = {k: [] for k in ("phi", "K", "alpha", "a", "U_D", "t", "dt_solid", "outer_its")}
    t = 0.0
    t0 = time.perf_counter()
    for _ in range(max_steps):
        d = sim.step(dt)
        t += d["dt_solid"]
        rec["phi"].append(phi)
        rec["K"].append(d["K"])
        rec["alpha"].append(d["alpha"])
        rec["a"].append(d["surface_area"] / volume)
        rec["U_D"].append(d["U_D"])
        rec["t"].append(t)
        rec["dt_solid"].append(d["dt_solid"])
        rec["outer_its"].append(d["outer_its"])
        phi = d["porosity"]
        if target_porosity is not None and phi >= target_porosity:
            break
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
    out = {k: np.array(v) for k, v in rec.items()}
    out["phi_end"] = phi
    out["wall_s"] = time.perf_counter() - t0
    return out

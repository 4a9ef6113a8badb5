"""Upscaled quantities of a dissolution run and their power-law fits --
TEST INFRASTRUCTURE ONLY (the same rule as the rest of ``oracle``: only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg use it).

Section 2.5 describes the whole domain of a dissolution run by its total
porosity phi, Darcy velocity U_D, permeability K, specific surface area a and
the correction factor alpha, and models K and alpha as power laws of phi;
Section 3.3 fits K = C phi^n (with two such laws, one before and one after
reactant breakthrough, for the wormhole regime) and alpha = C phi^m.

``run`` steps the oracle (Appendix D's bound on the solid step, deps_max)
and records, per step, the porosity at which that step's flow and transport
were solved (the mean fluid fraction at the step's start) beside the K, alpha,
a and U_D the step reports.  ``fit_power_law`` is ordinary least squares on
(log phi, log y) written out as the two-parameter normal equations;
``fit_two_power_laws`` tries every split of the points (each side keeping at
least ``min_points``) and keeps the one with the smallest summed squared
log residual.
"""
from __future__ import annotations

import math

import numpy as np

from . import step as _step


def fit_power_law(phi, y):
    """(C, n, rms) of y = C phi^n by least squares in logs: with X = log phi,
    Y = log y over m points, n = (m Sxy - Sx Sy) / (m Sxx - Sx^2),
    log C = (Sy - n Sx) / m; rms is the root mean square log residual."""
    X = [math.log(v) for v in phi]
    Y = [math.log(v) for v in y]
    m = len(X)
    if m < 2:
        raise ValueError("need two points")
    sx = sy = sxx = sxy = 0.0
    for a, b in zip(X, Y):
        sx += a
        sy += b
        sxx += a * a
        sxy += a * b
    den = m * sxx - sx * sx
    if den <= 0.0:
        raise ValueError("porosity does not vary")
    n = (m * sxy - sx * sy) / den
    logc = (sy - n * sx) / m
    ss = 0.0
    for a, b in zip(X, Y):
        r = b - (logc + n * a)
        ss += r * r
    return math.exp(logc), n, math.sqrt(ss / m)


def fit_two_power_laws(phi, y, min_points=3):
    """Best split into two power laws: (index of the first point of the second
    law, (C1, n1, rms1), (C2, n2, rms2)).  The points are taken in the order
    given (the run's order); the split minimises the total squared log residual."""
    m = len(phi)
    best = None
    for k in range(min_points, m - min_points + 1):
        f1 = fit_power_law(phi[:k], y[:k])
        f2 = fit_power_law(phi[k:], y[k:])
        ss = f1[2] ** 2 * k + f2[2] ** 2 * (m - k)
        if best is None or ss < best[0]:
            best = (ss, k, f1, f2)
    if best is None:
        raise ValueError("too few points for two laws")
    return best[1], best[2], best[3]


def run(prob, st, dt, steps, target_porosity=None):
    """Step the oracle up to ``steps`` times (until the porosity reaches
    ``target_porosity``, if given); returns a dict of per-step arrays: phi (mean
    eps at the step's start), K, alpha, a (surface area per volume), U_D, t (time
    at the step's end), dt_solid."""
    rec = {k: [] for k in ("phi", "K", "alpha", "a", "U_D", "t", "dt_solid")}
    t = 0.0
    vol = float(st.eps.size) * prob.dx ** 3
    for _ in range(steps):
        phi0 = float(np.mean(st.eps))
        d = _step(prob, st, dt)
        t += d["dt_solid"]
        rec["phi"].append(phi0)
        rec["K"].append(d["K"])
        rec["alpha"].append(d["alpha"])
        rec["a"].append(d["surface_area"] / vol)
        rec["U_D"].append(d["U_D"])
        rec["t"].append(t)
        rec["dt_solid"].append(d["dt_solid"])
        if target_porosity is not None and d["porosity"] >= target_porosity:
            break
    return {k: np.array(v) for k, v in rec.items()}

"""Reference scales and dimensionless groups of Section 2.5 / Section 3.

Pe = U L / D, Da = k_c / U (Ki = Da Pe), with the average pore velocity
U = U_D / phi and the pore length L = sqrt(c K / phi): c = 12 for the 2-D
micromodel (Section 3.2), c = 8 for the 3-D rock (Section 3.3).
"""
from __future__ import annotations

import math


def pore_length(K: float, phi: float, ndim: int) -> float:
    return math.sqrt((12.0 if ndim == 2 else 8.0) * K / phi)


def scales(K: float, phi: float, U_D: float, D: float, kc: float, ndim: int) -> dict:
    """(U, L, Pe, Da, Ki) from permeability K, porosity phi, Darcy velocity U_D."""
    U = U_D / phi
    L = pore_length(K, phi, ndim)
    Pe = U * L / D
    Da = kc / U
    return dict(U=U, L=L, Pe=Pe, Da=Da, Ki=Pe * Da)


def inlet_for(Pe: float, Da: float, K: float, phi: float, D: float, ndim: int):
    """Darcy (= inlet plug) velocity and reaction constant giving (Pe, Da)."""
    L = pore_length(K, phi, ndim)
    U = Pe * D / L
    return U * phi, Da * U


def pressure_drop_for(Pe: float, Da: float, K: float, phi: float, D: float, mu: float, L_D: float, ndim: int):
    """Pressure drop across L_D and reaction constant giving (Pe, Da) under a
    pressure drive: the Darcy velocity U_D = U phi of inlet_for, dP = mu U_D L_D / K
    (Section 2.5's permeability read backwards)."""
    U_D, kc = inlet_for(Pe, Da, K, phi, D, ndim)
    return mu * U_D * L_D / K, kc

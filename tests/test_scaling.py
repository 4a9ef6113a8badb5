"""Reference scales against the paper's Benchmark 3 worked example (Section 3.3):
Q = 8.33e-9 m3/s through a 1.7 mm-radius core, phi = 0.173, K = 16 D,
D = 7.5e-10 m2/s, k_c = 2.314e-4 m/s give U = 5.3e-3 m/s, L = 27 um,
Pe = 190 and Da = 4.4e-2 (printed to two significant figures)."""
import math

import pytest

from paper_2204_07019_amd import scaling

DARCY = 9.869233e-13


def test_ketton_worked_example():
    U_D = 8.33e-9 / (math.pi * 1.7e-3 ** 2)
    s = scaling.scales(K=16 * DARCY, phi=0.173, U_D=U_D, D=7.5e-10, kc=2.314e-4, ndim=3)
    assert s["U"] == pytest.approx(5.3e-3, abs=0.05e-3)
    assert s["L"] == pytest.approx(27e-6, abs=0.5e-6)
    assert s["Pe"] == pytest.approx(190, abs=5)
    assert s["Da"] == pytest.approx(4.4e-2, abs=0.05e-2)


def test_inverse_round_trip():
    for nd in (2, 3):
        ud, kc = scaling.inlet_for(Pe=10.0, Da=0.1, K=3e-11, phi=0.6, D=1e-9, ndim=nd)
        s = scaling.scales(K=3e-11, phi=0.6, U_D=ud, D=1e-9, kc=kc, ndim=nd)
        assert s["Pe"] == pytest.approx(10.0, rel=1e-12)
        assert s["Da"] == pytest.approx(0.1, rel=1e-12)


def test_micromodel_length_uses_factor_12():
    """Section 3.2: L = sqrt(12 K / phi) (phi = 0.45, K = 5.6e-10 m2)."""
    assert scaling.pore_length(5.6e-10, 0.45, 2) == pytest.approx(math.sqrt(12 * 5.6e-10 / 0.45))

"""The upscaling workload on the GPU against the oracle: the same dissolution
run (solid steps bounded by deps_max, Appendix D) recorded step by step --
porosity, permeability, correction factor, surface area, Darcy velocity,
simulated time -- and the power-law fits of K(phi) and alpha(phi) (Section
2.5; Section 3.3's fits) from each side's records by each side's fitter."""
import sys

import numpy as np
import pytest

from gpu_cases import gpu_sim, make_problem

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("model,precision", [(0, 0), (0, 1), (2, 1)])
def test_upscaling_run_matches_oracle(orc, model, precision):
    from oracle import upscaling as U
    from paper_2204_07019_amd import inputs
    from paper_2204_07019_amd import upscaling as G
    es = inputs.rsa_discs(96, 48, seed=5, rmin=5.0, rmax=9.0, porosity=0.6, gap=2.0, band=2)
    es = es.reshape((1,) + es.shape[-2:])
    # quasi-static stepping (Appendices A, B, D): the SIMPLE loop with a fixed
    # number of outer iterations on both sides (outer_tol 0), the solid step
    # set by deps_max
    prob = make_problem(es, dict(inputs.BASE_PARAMS, dx=5e-6, kc=1e-3), model=model, deps_max=0.02,
                        simple=1, outer_max=25, outer_tol=0.0, relax_u=0.7, relax_p=0.3, relax_c=1.0,
                        rtol_u=1e-12, rtol_p=1e-12, rtol_c=1e-12)
    dt, steps = 1e3, 10
    _say(f"upscaling 96x48 model {model} precision {precision}, {steps} steps")
    st = orc.initial_state(prob, es)
    ro = U.run(prob, st, dt, steps)
    sim = gpu_sim(prob, precision)
    sim.set_solid_fraction(es)
    rg = G.run(sim, dt, steps)
    sim.close()
    assert len(rg["phi"]) == len(ro["phi"]) == steps
    for k in ("phi", "K", "alpha", "a", "U_D", "t", "dt_solid"):
        err = np.max(np.abs(rg[k] - ro[k]) / np.abs(ro[k]))
        print(f"[parity] {k}: max rel {err:.2e}", flush=True)
        assert err < 1e-6, k
    assert ro["phi"][-1] > ro["phi"][0] + 1e-4
    assert np.all(ro["dt_solid"] < dt)
    for y in ("K", "alpha"):
        cg, ng, _ = G.fit_power_law(rg["phi"], rg[y])
        co, no, _ = U.fit_power_law(ro["phi"], ro[y])
        print(f"[parity] {y} = C phi^n: GPU n {ng:.6f}, oracle n {no:.6f}", flush=True)
        assert ng == pytest.approx(no, rel=1e-4, abs=1e-4)
        assert cg == pytest.approx(co, rel=1e-3)

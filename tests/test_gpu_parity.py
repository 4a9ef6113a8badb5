"""GPU (gfx950 HIP path, through the C ABI) against the FP64 oracle.

Parity bar: relative L2 <= 1e-6 on every face velocity, p, c, eps and the
change of eps, after N steps from the same seeded inputs (the solver
tolerances are tightened so the comparison measures the implementations,
not the stopping rule).  At full workload sizes, where the oracle cannot run
many steps, every stage's GPU output is checked against the oracle's own
discrete equations assembled from the same input state.
"""
import sys

import numpy as np
import pytest

from gpu_cases import gpu_sim, make_problem, rel_l2, run_both

pytestmark = pytest.mark.gpu

TIGHT = dict(rtol_u=1e-12, rtol_p=1e-12, rtol_c=1e-12)
BAR = 1e-6


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_07019_amd import vos
    vos.lib()


def _compare(st, g, eps0, tol=BAR):
    out = {k: rel_l2(g[k], getattr(st, k)) for k in ("ux", "uy", "p", "c", "eps")}
    if st.eps.shape[0] > 1:
        out["uz"] = rel_l2(g["uz"], st.uz)
    out["deps"] = rel_l2(g["eps"] - eps0, st.eps - eps0)
    for k, v in out.items():
        assert v <= tol, (k, v, out)
    return out


def test_post_20_steps_fp64(orc):
    """The 256x64 calcite-post channel (dx = 5 um, iVoS, FP64), 20 steps of 1 ms."""
    from paper_2204_07019_amd import inputs
    es, prm = inputs.workload("post")
    prob = make_problem(es, prm, model=0, **TIGHT)
    _say("post 256x64 iVoS fp64 20 steps")
    st, g, eps0, diags = run_both(es, prob, 1e-3, 20)
    r = _compare(st, g, eps0)
    _say(f"post rel L2 {r}")
    do, dg = diags[-1]
    assert abs(dg["acid_balance_rel"]) < 1e-9
    assert abs(dg["solid_balance_rel"]) < 1e-9
    assert dg["solid_rate"] == pytest.approx(do["solid_rate"], rel=1e-6)


def test_post_stagewise_one_step(orc):
    """Intermediate outputs of one step: momentum predictor, reaction rate, |grad eps|."""
    import oracle
    from paper_2204_07019_amd import inputs
    es, prm = inputs.workload("post")
    prob = make_problem(es, prm, model=0, **TIGHT)
    st = oracle.initial_state(prob, es)
    for _ in range(2):
        oracle.step(prob, st, 1e-3)
    sim = gpu_sim(prob)
    for k in ("eps", "ux", "uy", "p", "c"):
        sim.set(k, getattr(st, k))
    _say("post stagewise")
    d, it = oracle.step(prob, st, 1e-3, intermediates=True)
    sim.step(1e-3)
    assert rel_l2(sim.get_numpy("ustar_x"), it["ustar_x"]) < 1e-9
    assert rel_l2(sim.get_numpy("ustar_y"), it["ustar_y"]) < 1e-9
    assert rel_l2(sim.get_numpy("gmag"), it["gmag"]) < 1e-13
    assert rel_l2(sim.get_numpy("rbar"), it["rbar"]) < 1e-7
    sim.close()


@pytest.mark.parametrize("model", [0, 1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_models_and_precisions_2d(orc, model, precision):
    """iVoS / VoS-psi / VoS-psi' with FP64 and mixed (FP32 multigrid)
    pressure preconditioning, on a ragged 2-D grid with two grains."""
    from paper_2204_07019_amd import inputs
    es = inputs.rsa_discs(96, 40, seed=7, rmin=4, rmax=9, porosity=0.75)
    prm = dict(inputs.BASE_PARAMS, dx=5e-6)
    prob = make_problem(es, prm, model=model, **TIGHT)
    _say(f"rsa 96x40 model {model} precision {precision}")
    st, g, eps0, diags = run_both(es, prob, 2e-3, 6, precision=precision)
    _compare(st, g, eps0)


@pytest.mark.parametrize("shape", [(37, 23, 1), (24, 16, 12), (17, 9, 7)])
def test_ragged_and_3d(orc, shape):
    """Odd sizes (multigrid hierarchy cut short, Jacobi coarsest level) and 3-D."""
    from paper_2204_07019_amd import inputs
    nx, ny, nz = shape
    rng = np.random.default_rng(nx * 100 + ny)
    es = np.zeros((nz, ny, nx))
    es[:, ny // 4: 3 * ny // 4, nx // 3: nx // 3 + max(2, nx // 5)] = 1.0
    es[:, 1: ny // 4, nx // 2 + 1] = rng.uniform(0.3, 0.7)
    prm = dict(inputs.BASE_PARAMS, dx=5e-6)
    prob = make_problem(es, prm, model=0, **TIGHT)
    _say(f"ragged {shape}")
    st, g, eps0, diags = run_both(es, prob, 1e-3, 4, precision=1)
    _compare(st, g, eps0)


def test_empty_solid_and_fully_fluid(orc):
    """Degenerate geometries: no solid at all (no reaction, c -> c_in)."""
    from paper_2204_07019_amd import inputs
    es = np.zeros((1, 16, 32))
    prob = make_problem(es, dict(inputs.BASE_PARAMS, dx=5e-6), **TIGHT)
    _say("fully fluid 32x16")
    st, g, eps0, diags = run_both(es, prob, 1e-3, 3)
    for k in ("ux", "uy", "p", "c"):
        assert rel_l2(g[k], getattr(st, k)) < BAR
    assert np.all(g["eps"] == 1.0)
    assert diags[-1][1]["solid_rate"] == 0.0


def test_bad_inputs_raise(orc):
    from paper_2204_07019_amd import vos
    from paper_2204_07019_amd import inputs
    es = np.zeros((1, 8, 16))
    prob = make_problem(es, dict(inputs.BASE_PARAMS, dx=5e-6))
    sim = gpu_sim(prob)
    with pytest.raises(vos.VosError) as e:
        sim.step(1e-3)
    assert e.value.status == vos.VOS_ERR_STATE
    bad = es.copy()
    bad[0, 0, 0] = 1.5
    with pytest.raises(vos.VosError) as e:
        sim.set_solid_fraction(bad)
    assert e.value.status == vos.VOS_ERR_ARG
    sim.close()


def test_noconv_is_reported(orc):
    """maxit = 1 cannot reach the tolerance: the call says so (VOS_ERR_NOCONV)."""
    from paper_2204_07019_amd import vos, inputs
    es = inputs.calcite_post(64, 32, 20, 16, 6)
    prob = make_problem(es, dict(inputs.BASE_PARAMS, dx=5e-6), **TIGHT)
    sim = gpu_sim(prob, maxit_c=1)
    sim.set_solid_fraction(es)
    with pytest.raises(vos.VosError) as e:
        sim.step(1e-3)
    assert e.value.status == vos.VOS_ERR_NOCONV
    sim.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager(orc, precision):
    """Captured iteration chunks, replayed many times across steps with host
    synchronisations in between, give bitwise the same fields as plain launches."""
    from paper_2204_07019_amd import inputs
    es = inputs.rsa_discs(128, 64, seed=5, rmin=5, rmax=12, porosity=0.7)
    prob = make_problem(es, dict(inputs.BASE_PARAMS, dx=5e-6), rtol_u=1e-9, rtol_p=1e-9, rtol_c=1e-9)
    out = []
    for graphs in (0, 1):
        _say(f"graph replay precision {precision} graphs {graphs}")
        sim = gpu_sim(prob, precision, use_graphs=graphs, check_every=4)
        sim.set_solid_fraction(es)
        for _ in range(4):
            sim.step(1e-3)
        out.append({k: sim.get_numpy(k) for k in ("ux", "uy", "p", "c", "eps")})
        sim.close()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k

"""Shared drivers for the GPU parity tests: run the HIP path and the oracle
on the same seeded inputs."""
import numpy as np

import oracle
from paper_2204_07019_amd import inputs


def make_problem(es, prm, model=0, nz=None, **tol):
    nz_, ny, nx = es.shape
    kw = dict(prm)
    kw.update(model=model)
    kw.update(tol)
    return oracle.Problem(nx=nx, ny=ny, nz=nz_, **kw)


def gpu_params(prob):
    """vos_params of an oracle problem (same names)."""
    from paper_2204_07019_amd import vos
    return {k: getattr(prob, k) for k, _ in vos._Params._fields_}


def gpu_sim(prob, precision=0, **opt_overrides):
    from paper_2204_07019_amd import vos
    params = gpu_params(prob)
    o = vos.Opts(rtol_u=prob.rtol_u, rtol_p=prob.rtol_p, rtol_c=prob.rtol_c,
                 maxit_u=prob.maxit_u, maxit_p=min(prob.maxit_p, 5000), maxit_c=prob.maxit_c,
                 precision=precision, deps_max=prob.deps_max, simple=prob.simple,
                 outer_max=prob.outer_max, outer_tol=prob.outer_tol, relax_u=prob.relax_u,
                 relax_p=prob.relax_p, relax_c=prob.relax_c, solid_dt=prob.solid_dt)
    for k, v in opt_overrides.items():
        setattr(o, k, v)
    return vos.Sim(prob.nx, prob.ny, prob.nz, prob.dx, params, o)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def run_both(es, prob, dt, nsteps, precision=0, **opt):
    """Advance the oracle and the GPU nsteps from the same initial state;
    return (oracle state, gpu fields dict, initial eps, per-step diags)."""
    st = oracle.initial_state(prob, es)
    eps0 = st.eps.copy()
    sim = gpu_sim(prob, precision, **opt)
    sim.set_solid_fraction(es)
    diags = []
    for _ in range(nsteps):
        do = oracle.step(prob, st, dt)
        dg = sim.step(dt)
        diags.append((do, dg))
    g = {k: sim.get_numpy(k) for k in ("eps", "ux", "uy", "uz", "p", "c")}
    sim.close()
    return st, g, eps0, diags

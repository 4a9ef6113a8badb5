"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle (oracle/vos_oracle.c) against something other than
itself: closed-form solutions, exact discrete identities of the method,
convergence orders, brute-force dense solves, textbook formulas, and the
paper's printed numbers.  None of them needs a GPU.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ helpers

def _channel(orc, ny, eps, k0, nx_factor=6, H=80e-6, nsteps=400, **kw):
    """Run a uniform-porosity channel with plug inflow to its steady state."""
    nx = nx_factor * ny
    dx = H / ny
    prob = orc.Problem(nx=nx, ny=ny, dx=dx, kc=0.0, k0=k0, u_in=1e-4, rtol_u=1e-13,
                       rtol_p=1e-13, rtol_c=1e-10, **kw)
    st = orc.initial_state(prob, np.full((1, ny, nx), 1.0 - eps))
    dt = H * H * prob.rho / prob.mu / 50.0
    for _ in range(nsteps):
        u0 = st.ux.copy()
        p0 = st.p.copy()
        orc.step(prob, st, dt)
        du = np.abs(st.ux - u0).max() / np.abs(st.ux).max()
        dp = np.abs(st.p - p0).max() / np.abs(st.p).max()
        if du < 1e-12 and dp < 1e-11:
            break
    y = (np.arange(ny) + 0.5) * dx
    return st.ux[0, :, nx // 2], y, H, st, prob


# ------------------------------------------------- momentum + pressure

def test_poiseuille_second_order(orc):
    """Plane Poiseuille flow u = 6 U (y/H)(1 - y/H) (eps = 1: Eq. momentumDBS
    reduces to Stokes); the no-slip ghost makes the scheme O(dx^2)."""
    errs = []
    for ny in (8, 16):
        prof, y, H, st, prob = _channel(orc, ny, eps=1.0, k0=1e-15)
        exact = 6 * prob.u_in * (y / H) * (1 - y / H)
        errs.append(np.abs(prof - exact).max() / exact.max())
        # mean flux equals the inlet flux (continuity, Eq. contDBSQS)
        assert abs(prof.mean() - prob.u_in) < 1e-9 * prob.u_in
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 3.5, errs


def test_poiseuille_pressure_gradient(orc):
    """Fully developed pressure gradient dp/dx = -12 mu U / H^2 (to O(dx^2))."""
    prof, y, H, st, prob = _channel(orc, 16, eps=1.0, k0=1e-15)
    nx = prob.nx
    dx = prob.dx
    row = st.p[0, prob.ny // 2, :]
    g = (row[2 * nx // 3] - row[nx // 3]) / ((2 * nx // 3 - nx // 3) * dx)
    exact = -12 * prob.mu * prob.u_in / H ** 2
    assert abs(g - exact) / abs(exact) < 2e-2


def test_brinkman_channel_kozeny_carman(orc):
    """Brinkman channel with uniform eps: (mu/eps) u'' - (mu/k) u = -G with
    k = k0 eps^3 / (1-eps)^2 (Eq. perm).  Closed form
    u = (G k / mu) [1 - cosh((y - H/2)/l) / cosh(H/(2 l))], l = sqrt(k/eps)."""
    eps, k0 = 0.5, 4e-10
    errs = []
    for ny in (8, 16):
        prof, y, H, st, prob = _channel(orc, ny, eps=eps, k0=k0)
        k = k0 * eps ** 3 / (1 - eps) ** 2
        l = np.sqrt(k / eps)
        shape = 1 - np.cosh((y - H / 2) / l) / np.cosh(H / (2 * l))
        exact = prob.u_in * shape / (1 - (2 * l / H) * np.tanh(H / (2 * l)))
        errs.append(np.abs(prof - exact).max() / exact.max())
    assert errs[1] < 1.2e-2
    assert errs[0] / errs[1] > 2.8, errs


# --------------------------------------------------------- transport

def test_reactive_plane_first_order(orc):
    """1-D diffusion from the inlet (c_in) to a reactive solid plane at L:
    flux J = c_in / (1/k_c + L/D).  The iVoS interface is one cell wide, so
    the scheme converges at first order."""
    Lf, D, kc, cin = 100e-6, 1e-9, 1e-5, 10.0
    Jex = cin / (1 / kc + Lf / D)
    errs = []
    for m in (10, 20, 40):
        dx = Lf / m
        nx = m + m // 2
        prob = orc.Problem(nx=nx, ny=2, dx=dx, kc=kc, D=D, u_in=0.0, c_in=cin,
                           rtol_u=1e-13, rtol_p=1e-13, rtol_c=1e-14)
        es = np.zeros((1, 2, nx))
        es[:, :, m:] = 1.0
        st = orc.initial_state(prob, es)
        d = orc.step(prob, st, 1e-3)
        J = d["acid_consumed"] / (2 * dx * dx)
        errs.append(abs(J - Jex) / Jex)
        # diffusion only: the fluid profile is linear in x up to the reacting cells
        row = st.c[0, 0, : m - 3]
        assert np.abs(np.diff(row, 2)).max() < 1e-9 * cin
    assert errs[-1] < 0.02
    assert 1.8 < errs[0] / errs[1] < 2.3 and 1.8 < errs[1] / errs[2] < 2.3, errs


def test_uniform_concentration_is_steady(orc):
    """With no reaction, uniform c = c_in satisfies the transport equation
    exactly (conservative convection of a divergence-free flux + diffusion)."""
    prob = orc.Problem(nx=24, ny=12, kc=0.0, rtol_c=1e-14, rtol_u=1e-13, rtol_p=1e-13)
    es = np.zeros((1, 12, 24))
    es[0, 4:8, 8:14] = 1.0
    st = orc.initial_state(prob, es)
    for _ in range(3):
        orc.step(prob, st, 1e-3)
    st.c[:] = prob.c_in
    orc.step(prob, st, 1e-3)
    assert np.abs(st.c - prob.c_in).max() < 1e-9 * prob.c_in


def test_alpha_is_inverse_porosity_for_uniform_concentration(orc):
    """The correction factor alpha = sum c |grad eps| V / (a sum eps c V) with
    a = sum |grad eps| V / V_domain (Section 2.5): for a uniform c it is
    V_domain / sum eps V = 1 / phi, whatever the geometry and the value of c.
    A c missing from one of the sums (c_in != 1), an area normalised by
    anything but the domain volume, or an eps weighting of another field
    fails here.  No reaction (kc = 0) keeps c uniform and eps fixed."""
    for nz, cin in ((1, 2.5), (1, 0.4), (6, 3.0)):
        prob = orc.Problem(nx=24, ny=12, nz=nz, kc=0.0, c_in=cin, rtol_c=1e-14, rtol_u=1e-13, rtol_p=1e-13)
        es = np.zeros((nz, 12, 24))
        es[:, 4:8, 8:14] = 1.0
        es[:, 3, 8:14] = 0.35          # partial cells: |grad eps| varies along the interface
        es[:, 2:9, 15] = 0.6
        st = orc.initial_state(prob, es)
        for _ in range(2):
            orc.step(prob, st, 1e-3)
        st.c[:] = cin
        d = orc.step(prob, st, 1e-3)
        phi = float(np.mean(st.eps))
        assert d["alpha"] == pytest.approx(1.0 / phi, rel=1e-9), (nz, cin)
        assert d["porosity"] == pytest.approx(phi, rel=1e-14)


# ------------------------------------------------------- reaction rate

def _plane(orc, model, m=6, nx=16, ny=4, eps_front=None, c=3.0):
    prob = orc.Problem(nx=nx, ny=ny, model=model, kc=2e-4)
    es = np.zeros((1, ny, nx))
    es[:, :, m:] = 1.0
    eps = orc.eps_from_solid(prob, es)
    if eps_front is not None:
        eps[:, :, m] = eps_front
    cc = np.full(prob.cell_shape, c)
    return prob, eps, cc


def test_plane_front_ivos_exact(orc):
    """Frozen uniform c on a flat solid plane: iVoS gives total rate
    k_c c A (1 - eps_min) exactly, all of it in the first solid cell, i.e.
    the interface recedes at w = V_m k_c c (Eq. Ws with R = k_c c)."""
    prob, eps, c = _plane(orc, 0)
    rbar, sink, gmag, lam, eps1 = orc.reaction(prob, 1e-3, eps, c)
    A = prob.ny * prob.dx ** 2
    V = prob.dx ** 3
    total = rbar.sum() * V
    assert total == pytest.approx(prob.kc * 3.0 * A * (1 - prob.eps_min), rel=1e-13)
    assert np.allclose(rbar[:, :, 6], prob.kc * 3.0 * (1 - prob.eps_min) / prob.dx, rtol=1e-13)
    mask = np.ones_like(rbar, dtype=bool)
    mask[:, :, 6] = False
    assert np.abs(rbar[mask]).max() < 1e-13 * rbar.max()
    # the acid sink equals the solid rate globally (Eq. RfiVoS conservative term sums to 0)
    assert sink.sum() == pytest.approx(total, rel=1e-13)
    # front displacement per step = Vm k_c c dt (1 - eps_min)
    dvol = (eps1 - eps).sum() * V
    assert dvol / A == pytest.approx(prob.Vm * prob.kc * 3.0 * 1e-3 * (1 - prob.eps_min), rel=1e-12)


def test_plane_front_moves_at_vm_kc_c(orc):
    """Over many frozen-c steps the iVoS front advances at exactly
    V_m k_c c (1 - eps_min) per unit time while it stays flat, including
    while cells are partially dissolved."""
    prob, eps, c = _plane(orc, 0, m=5, nx=20)
    dt = 2.0  # large step so the front crosses cells
    V = prob.dx ** 3
    A = prob.ny * prob.dx ** 2
    vol0 = ((1 - eps) * V).sum()
    rate = prob.Vm * prob.kc * 3.0 * (1 - prob.eps_min)
    n = 0
    for n in range(1, 40):
        rbar, sink, gmag, lam, eps_new = orc.reaction(prob, dt, eps, c)
        unclipped = eps + dt * prob.Vm * rbar
        clip = ((unclipped - eps_new) * V).sum()
        eps = eps_new
        if abs(clip) > 0:
            break
        vol = ((1 - eps) * V).sum()
        assert (vol0 - vol) / A == pytest.approx(rate * dt * n, rel=1e-10)
    assert n > 3


def test_plane_front_psi_prime_exact_and_psi_factor(orc):
    """VoS-psi' fits lambda so that the total reactive area sum psi|grad eps|V
    equals sum |grad eps| V (Section 2.4): same total rate as iVoS.  VoS-psi
    (lambda = 4) under-reacts by sum 4 eps(1-eps)|g| / sum |g|."""
    prob, eps, c = _plane(orc, 2, eps_front=0.4)
    rb2, _, g, lam, _ = orc.reaction(prob, 1e-3, eps, c)
    V = prob.dx ** 3
    area = (g * V).sum()
    assert (rb2 * V).sum() == pytest.approx(prob.kc * 3.0 * area, rel=1e-13)
    assert lam == pytest.approx(g.sum() / (g * eps * (1 - eps)).sum(), rel=1e-14)
    prob1, _, _ = _plane(orc, 1, eps_front=0.4)
    rb1, _, _, lam1, _ = orc.reaction(prob1, 1e-3, eps, c)
    assert lam1 == 4.0
    factor = (4 * eps * (1 - eps) * g).sum() / g.sum()
    assert (rb1 * V).sum() == pytest.approx(prob.kc * 3.0 * area * factor, rel=1e-13)
    # central differences: the plane's area is (1 - eps_min)... spread over two cells
    prob_s, eps_s, c_s = _plane(orc, 2)
    _, _, g_s, _, _ = orc.reaction(prob_s, 1e-3, eps_s, c_s)
    assert (g_s * V).sum() == pytest.approx(prob.ny * prob.dx ** 2 * (1 - prob.eps_min), rel=1e-13)


@pytest.mark.parametrize("nz", [1, 5])
def test_isolated_remnant(orc, nz):
    """A single partially dissolved cell surrounded by fluid.  iVoS: the
    2 n_d faces carry half-normals into it, Rbar = n_d k_c c (1 - eps_P)/dx.
    Centred VoS-psi: grad eps = 0 there, so Rbar = 0 -- the incomplete
    dissolution of Section 2.4."""
    n = 5
    ny = n
    prob = orc.Problem(nx=n, ny=ny, nz=nz, kc=3e-4, model=0)
    eps = np.ones(prob.cell_shape)
    k0 = nz // 2
    eps[k0, 2, 2] = 0.35
    c = np.full(prob.cell_shape, 2.0)
    rbar, _, _, _, _ = orc.reaction(prob, 1e-3, eps, c)
    nd = 2 if nz == 1 else 3
    assert rbar[k0, 2, 2] == pytest.approx(nd * prob.kc * 2.0 * (1 - 0.35) / prob.dx, rel=1e-14)
    other = rbar.copy()
    other[k0, 2, 2] = 0
    assert np.abs(other).max() < 1e-14 * rbar[k0, 2, 2]
    prob_psi = orc.Problem(nx=n, ny=ny, nz=nz, kc=3e-4, model=1)
    rb, _, _, _, _ = orc.reaction(prob_psi, 1e-3, eps, c)
    assert rb[k0, 2, 2] == 0.0


def test_vanleer_textbook(orc):
    """The face value equals phi_C + psi(r)/2 (phi_D - phi_C) with van Leer's
    limiter psi(r) = (r + |r|)/(1 + |r|), r = (phi_C - phi_U)/(phi_D - phi_C)."""
    rng = np.random.default_rng(5)
    for _ in range(2000):
        u, cc, d = rng.normal(size=3)
        r = (cc - u) / (d - cc)
        psi = (r + abs(r)) / (1 + abs(r))
        assert orc.vanleer_face(u, cc, d) == pytest.approx(cc + 0.5 * psi * (d - cc), rel=1e-12, abs=1e-14)
    # linear data -> midpoint (second order); extrema and ties -> upwind
    assert orc.vanleer_face(1.0, 2.0, 3.0) == 2.5
    assert orc.vanleer_face(1.0, 3.0, 2.0) == 3.0
    assert orc.vanleer_face(2.0, 2.0, 5.0) == 2.0
    assert orc.vanleer_face(1.0, 2.0, 2.0) == 2.0


# ------------------------------------------------ linear systems (16^2)

def _random_state(orc, nx=16, ny=16, nz=1, seed=3, steps=2, model=0):
    from paper_2204_07019_amd import inputs
    rng = np.random.default_rng(seed)
    es = np.zeros((nz, ny, nx))
    es[:, 4:11, 5:10] = 1.0
    es[:, 6:8, 11:13] = rng.uniform(0.2, 0.8)
    prob = orc.Problem(nx=nx, ny=ny, nz=nz, model=model, rtol_u=1e-13, rtol_p=1e-13, rtol_c=1e-13)
    st = orc.initial_state(prob, es)
    for _ in range(steps):
        orc.step(prob, st, 1e-3)
    return prob, st


@pytest.mark.parametrize("which", [0, 1, 3, 4])
def test_dense_solves_16x16(orc, which):
    """The oracle's Krylov solvers reproduce numpy's dense LU solution of the
    assembled 16x16 systems (momentum x/y, pressure, transport)."""
    prob, st = _random_state(orc)
    sten, rhs, dims = orc.assemble(prob, st, 1e-3, which)
    A = orc.stencil_to_dense(sten, dims)
    x_dense = np.linalg.solve(A, rhs)
    kind = 1 if which == 4 else 0
    x, rc, its, rr = orc.solve_stencil(sten, dims, rhs, kind=kind, rtol=1e-14)
    assert rc == 0
    assert np.linalg.norm(x - x_dense) <= 1e-9 * np.linalg.norm(x_dense)


@pytest.mark.parametrize("which", [0, 1, 3])
def test_symmetric_systems_are_spd(orc, which):
    """Momentum (row-scaled by eps_f) and pressure matrices are symmetric
    positive definite (Cholesky succeeds)."""
    prob, st = _random_state(orc)
    sten, rhs, dims = orc.assemble(prob, st, 1e-3, which)
    A = orc.stencil_to_dense(sten, dims)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    # Jacobi-scale before factorising: the coefficients span ~1e18
    d = 1 / np.sqrt(np.diag(A))
    np.linalg.cholesky(A * d[:, None] * d[None, :])


def test_pressure_rows_annihilate_constants(orc):
    """Rows of cells without an outlet face sum to zero (a pure flux balance)."""
    prob, st = _random_state(orc)
    sten, rhs, dims = orc.assemble(prob, st, 1e-3, 3)
    A = orc.stencil_to_dense(sten, dims)
    s = A.sum(axis=1).reshape(prob.cell_shape)
    assert np.abs(s[:, :, :-1]).max() <= 1e-12 * np.abs(np.diag(A)).max()
    assert (s[:, :, -1] > 0).all()


def test_transport_is_m_matrix_like(orc):
    """Upwind convection + diffusion: positive diagonal, non-positive
    off-diagonals in fluid rows."""
    prob, st = _random_state(orc)
    sten, rhs, dims = orc.assemble(prob, st, 1e-3, 4)
    assert (sten[0] > 0).all()
    fluid = (st.eps.ravel() == 1.0)
    assert (sten[1:, fluid] <= 1e-30).all()


# --------------------------------------------------------- conservation

@pytest.mark.parametrize("model", [0, 1, 2])
@pytest.mark.parametrize("nz", [1, 6])
def test_conservation(orc, model, nz):
    """Solid volume and acid moles balance to 1e-10 relative over full steps
    (the acid balance closes to the transport solve's tolerance)."""
    n = 16 if nz == 1 else 8
    es = np.zeros((nz, n, 2 * n))
    es[:, n // 4:n - n // 4, 6:12] = 1.0
    if nz > 1:
        es[:2, :, :] = 0.0
    assert es.sum() > 0
    prob = orc.Problem(nx=2 * n, ny=n, nz=nz, model=model, rtol_u=1e-13, rtol_p=1e-13, rtol_c=1e-14)
    st = orc.initial_state(prob, es)
    for _ in range(3):
        d = orc.step(prob, st, 1e-3)
        assert abs(d["acid_balance_rel"]) < 1e-10
        assert abs(d["solid_balance_rel"]) < 1e-10
        assert d["solid_rate"] > 0
        assert d["acid_consumed"] == pytest.approx(prob.zeta * d["solid_rate"], rel=1e-12)


# ------------------------------------------------ paper's printed numbers

def test_r_omega_reproduces_table(orc):
    """R_Omega = rho_s dphi / (M_w dt) (Section 3.3) maps the porosities of
    the poroPerm table onto the reactionRate table."""
    with open(os.path.join(GOLDEN, "ketton_tables.json")) as f:
        g = json.load(f)
    rho_s, M_w = g["rho_s_kg_m3"], g["M_w_kg_mol"]
    for key in ("simulation", "experiment"):
        phi = g["porosity"][key]
        for i, printed in enumerate(g["R_omega_mol_m3_s"][key]):
            r = orc.r_omega(rho_s, M_w, phi[i + 1] - phi[i], g["interval_s"])
            assert abs(r - printed) <= 0.0101, (key, i, r, printed)


# ------------------------------------------- largest change of eps (App. D)

def test_solid_step_limit(orc):
    """Appendix D holds the largest change of the fluid fraction per step to
    deps_max.  With the limit binding, the step's solves and rates are those
    of the unlimited step, the change of eps is the unlimited change scaled by
    dt_solid / dt in every cell that neither run clips, and the largest change
    equals the limit; a limit above the largest change leaves the step alone."""
    import copy
    import dataclasses
    prob, st = _random_state(orc, steps=2)
    dt = 1e-3
    e0 = st.eps.copy()
    a, b, c = copy.deepcopy(st), copy.deepcopy(st), copy.deepcopy(st)
    d0 = orc.step(prob, a, dt)
    assert d0["dt_solid"] == dt and d0["max_deps"] > 0
    lim = 0.25 * d0["max_deps"]
    d1 = orc.step(dataclasses.replace(prob, deps_max=lim), b, dt)
    assert 0 < d1["dt_solid"] < dt
    assert d1["solid_rate"] == d0["solid_rate"] and d1["it_p"] == d0["it_p"]
    free = (a.eps > prob.eps_min) & (a.eps < 1.0) & (b.eps > prob.eps_min) & (b.eps < 1.0)
    assert free.sum() > 0
    # eps is O(1): its change is known to a few units of 2^-52 after eps^n is subtracted
    np.testing.assert_allclose((b.eps - e0)[free], (a.eps - e0)[free] * (d1["dt_solid"] / dt),
                               rtol=1e-12, atol=4 * 2.0 ** -52)
    assert d1["max_deps"] == pytest.approx(lim, rel=1e-12)
    assert abs(d1["solid_balance_rel"]) < 1e-10
    d2 = orc.step(dataclasses.replace(prob, deps_max=4 * d0["max_deps"]), c, dt)
    assert d2["dt_solid"] == dt and np.array_equal(c.eps, a.eps)

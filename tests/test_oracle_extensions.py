"""Pins of the oracle's deferred van Leer correction, its flow diagnostics and
of the options beyond the single projection pass (pressure drive, momentum
convection, the SIMPLE loop of Appendices A-B, the transient terms of
Section 2.2, the VoS-psi variants of Section 2.4).

Every expected value here comes from a closed form of the continuous or the
discrete problem derived by hand for the specific field of the test, from a
convergence order, from a textbook formula written in a different form than
the oracle's, or from an exact identity between two independent outputs --
never from re-running the oracle's own expression.
"""
import copy
import dataclasses
import math

import numpy as np
import pytest


# ------------------------------------------------------------ helpers

def _flat_state(orc, prob, eps=1.0):
    es = np.full(prob.cell_shape, 1.0 - eps)
    return orc.initial_state(prob, es)


def _van_leer_psi_form(phi_u, phi_c, phi_d):
    """Correction to the upwind value in the textbook limiter form:
    0.5 psi(r) (phi_D - phi_C), psi(r) = (r + |r|) / (1 + |r|),
    r = (phi_C - phi_U) / (phi_D - phi_C); 0 when phi_D = phi_C."""
    den = phi_d - phi_c
    if den == 0.0:
        return 0.0
    r = (phi_c - phi_u) / den
    return 0.5 * (r + abs(r)) / (1 + abs(r)) * den


# ---------------------------------------------- deferred van Leer correction

def test_deferred_correction_stencil_both_signs(orc):
    """Transport right-hand side on a prescribed velocity field of random sign
    on every interior face (no diffusion, no reaction, c_in = 0): each cell's
    right-hand side is minus the sum over its interior faces of the outward
    flux times the van Leer correction taken on the upwind (C), downwind (D)
    and far-upwind (U) cells along that face's velocity, with U := C where the
    far-upwind cell falls outside the grid (zero-gradient ghost) -- checked
    face by face against the limiter written in its psi(r) form."""
    nx, ny, nz = 7, 5, 4
    prob = orc.Problem(nx=nx, ny=ny, nz=nz, D=0.0, kc=0.0, c_in=0.0)
    st = _flat_state(orc, prob)
    rng = np.random.default_rng(17)
    for name in ("ux", "uy", "uz"):
        a = getattr(st, name)
        a[:] = rng.normal(scale=1e-4, size=a.shape)
    st.uy[:, [0, ny], :] = 0.0          # no flow through the walls
    st.uz[[0, nz], :, :] = 0.0
    st.c[:] = rng.uniform(0.0, 10.0, size=st.c.shape)
    sten, rhs, dims = orc.assemble(prob, st, 1e-3, 4)
    c = st.c
    S = prob.dx ** 2
    expect = np.zeros(prob.cell_shape)
    n = (nz, ny, nx)
    for d, u in ((2, st.uz), (1, st.uy), (0, st.ux)):     # axes of (z, y, x) arrays
        ax = {0: 2, 1: 1, 2: 0}[d]
        for idx in np.ndindex(u.shape):
            q = idx[ax]
            if q == 0 or q == n[ax]:
                continue                       # boundary faces carry no correction
            lo = list(idx); lo[ax] -= 1; lo = tuple(lo)
            hi = idx
            vel = u[idx]
            if vel >= 0.0:
                C_, D_ = lo, hi
                U_ = list(lo); U_[ax] -= 1
            else:
                C_, D_ = hi, lo
                U_ = list(hi); U_[ax] += 1
            U_ = tuple(U_)
            phi_u = c[U_] if 0 <= U_[ax] < n[ax] else c[C_]
            corr = _van_leer_psi_form(phi_u, c[C_], c[D_])
            # outward flux of the lower cell is +S u, of the upper cell -S u
            expect[lo] -= S * vel * corr
            expect[hi] -= -S * vel * corr
    np.testing.assert_allclose(rhs.reshape(prob.cell_shape), expect, rtol=1e-12,
                               atol=1e-12 * np.abs(expect).max())
    # the implicit part is pure upwind: the diagonal is the sum of the outflows
    out = np.zeros(prob.cell_shape)
    for d, u in ((2, st.uz), (1, st.uy), (0, st.ux)):
        ax = {0: 2, 1: 1, 2: 0}[d]
        sl_lo = [slice(None)] * 3; sl_lo[ax] = slice(0, -1)
        sl_hi = [slice(None)] * 3; sl_hi[ax] = slice(1, None)
        out += np.maximum(-S * u[tuple(sl_lo)], 0.0) + np.maximum(S * u[tuple(sl_hi)], 0.0)
    # the outlet face's flux enters whatever its sign (zero-gradient c_f = c_P)
    out[:, :, -1] += np.minimum(S * st.ux[:, :, -1], 0.0)
    np.testing.assert_allclose(sten[0].reshape(prob.cell_shape), out, rtol=1e-12,
                               atol=1e-14 * np.abs(out).max())


def test_advection_diffusion_truncation_is_second_order(orc):
    """The steady 1-D advection-diffusion solution c = exp(Pe x / L) put into
    the transport rows with the correction lagged on itself (the converged
    deferred-correction scheme) leaves a residual per unit volume that falls
    as dx^2 in the interior: van Leer on a smooth monotone profile is second
    order (a missing or misplaced correction leaves first order)."""
    L, U, Pe = 1e-4, 1e-4, 5.0
    D = U * L / Pe
    errs = []
    for nx in (20, 40, 80):
        dx = L / nx
        prob = orc.Problem(nx=nx, ny=1, dx=dx, D=D, kc=0.0, u_in=U, c_in=1.0)
        st = _flat_state(orc, prob)
        st.ux[:] = U
        x = (np.arange(nx) + 0.5) * dx
        st.c[0, 0, :] = np.exp(Pe * x / L)
        sten, rhs, dims = orc.assemble(prob, st, 1e-3, 4)
        A = orc.stencil_to_dense(sten, dims)
        res = (A @ st.c.ravel() - rhs) / dx ** 3
        k = nx // 10
        errs.append(np.abs(res[k:nx - k]).max())
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.3, errs


# ------------------------------------------ Darcy slab: K and both drives

@pytest.mark.parametrize("three_d", [False, True])
@pytest.mark.parametrize("drive", [0, 1])
def test_darcy_slab_permeability(orc, drive, three_d):
    """Uniform porosity in a one-cell-wide slab (ny = 1; in 3-D two layers,
    nz = 2): the steady flow is uniform, u = -K_eff dp/dx, with the
    Kozeny-Carman permeability k = k0 eps^3/(1-eps)^2 in series with the
    no-slip walls' mirrored ghosts (2 mu u / dx^2 per wall side, n_w wall
    sides): 1/K_eff = 1/k + 2 n_w / (eps dx^2).  The K diagnostic returns
    K_eff, U_D the inlet flux per area, under the inlet velocity and the inlet
    pressure drive alike."""
    eps, k0, dx, nx = 0.4, 1e-12, 5e-6, 24
    nd3 = three_d
    prob = orc.Problem(nx=nx, ny=1, nz=2 if nd3 else 1, dx=dx, k0=k0, kc=0.0, u_in=2e-5, drive=drive,
                       p_in=0.5, p_out=0.1, rtol_u=1e-14, rtol_p=1e-14, rtol_c=1e-12)
    st = _flat_state(orc, prob, eps)
    d = None
    for _ in range(60):
        u0 = st.ux.copy()
        d = orc.step(prob, st, 1.0)
        if np.abs(st.ux - u0).max() <= 1e-15 * np.abs(st.ux).max():
            break
    k = k0 * eps ** 3 / (1 - eps) ** 2
    if nd3:
        # each x-face of a 2-layer slab: two y wall ghosts, one z wall ghost and
        # one z neighbour with the same velocity (no contribution)
        n_w = 3
    else:
        n_w = 2
    K_eff = 1.0 / (1.0 / k + 2 * n_w / (eps * dx ** 2))
    assert d["K"] == pytest.approx(K_eff, rel=1e-10)
    u = st.ux
    assert np.ptp(u) <= 1e-10 * np.abs(u).max()
    if drive == 0:
        assert d["U_D"] == pytest.approx(prob.u_in, rel=1e-14)
    else:
        L = nx * dx
        assert d["U_D"] == pytest.approx(K_eff * (prob.p_in - prob.p_out) / (prob.mu * L), rel=1e-10)
        assert d["dP"] == pytest.approx(prob.p_in - prob.p_out, rel=1e-15)


def test_pressure_drive_linear_pressure(orc):
    """Under the inlet pressure drive a uniform Darcy slab carries a linear
    pressure from p_in at the inlet face to p_out at the outlet face."""
    eps, nx, dx = 0.5, 16, 5e-6
    prob = orc.Problem(nx=nx, ny=1, dx=dx, k0=1e-12, kc=0.0, drive=1, p_in=2.0, p_out=0.0,
                       rtol_u=1e-14, rtol_p=1e-14)
    st = _flat_state(orc, prob, eps)
    for _ in range(60):
        orc.step(prob, st, 1.0)
    x = (np.arange(nx) + 0.5) * dx
    exact = prob.p_in + (prob.p_out - prob.p_in) * x / (nx * dx)
    np.testing.assert_allclose(st.p[0, 0], exact, rtol=1e-10, atol=1e-12)


# ------------------------------------------------- 3-D closed form: duct

def _duct_exact(yc, zc, a, b, mu, G, nterms=60):
    """Fully developed Stokes flow in a rectangular duct |y| < a, |z| < b
    under the pressure gradient -G (the classical Fourier series)."""
    u = np.zeros((len(zc), len(yc)))
    Y, Z = np.meshgrid(yc, zc)
    for n in range(1, 2 * nterms, 2):
        k = n * math.pi / (2 * a)
        u += ((-1) ** ((n - 1) // 2) / n ** 3 *
              (1 - np.cosh(k * Z) / np.cosh(k * b)) * np.cos(k * Y))
    return 16 * a * a * G / (mu * math.pi ** 3) * u


def _duct_mean(a, b, mu, G, nterms=60):
    s = sum(math.tanh(n * math.pi * b / (2 * a)) / n ** 5 for n in range(1, 2 * nterms, 2))
    return G * a * a / (3 * mu) * (1 - 192 * a / (math.pi ** 5 * b) * s)


@pytest.mark.slow
def test_square_duct_3d_second_order(orc):
    """3-D Stokes flow (eps = 1) through a square duct with no-slip walls on
    all four sides: the developed profile at mid-length matches the Fourier
    series of the duct at second order, and carries the inlet flux."""
    H = 60e-6
    errs = []
    for m in (6, 12):
        dx = H / m
        nx = 4 * m
        prob = orc.Problem(nx=nx, ny=m, nz=m, dx=dx, kc=0.0, k0=1e-15, u_in=1e-4,
                           rtol_u=1e-12, rtol_p=1e-12, rtol_c=1e-10)
        st = _flat_state(orc, prob)
        dt = H * H * prob.rho / prob.mu / 20.0
        for _ in range(300):
            u0 = st.ux.copy()
            orc.step(prob, st, dt)
            if np.abs(st.ux - u0).max() < 1e-11 * np.abs(st.ux).max():
                break
        prof = st.ux[:, :, nx // 2]
        a = b = H / 2
        yc = (np.arange(m) + 0.5) * dx - a
        G = prob.u_in / _duct_mean(a, b, prob.mu, 1.0)
        exact = _duct_exact(yc, yc, a, b, prob.mu, G)
        errs.append(np.abs(prof - exact).max() / exact.max())
        assert abs(prof.mean() - prob.u_in) < 1e-8 * prob.u_in
    assert errs[1] < 2e-2
    assert errs[0] / errs[1] > 3.3, errs


# ---------------------------------------------------- momentum convection

def _conv_rhs_difference(orc, prob, st, which):
    on = dataclasses.replace(prob, convection=1)
    _, b_on, dims = orc.assemble(on, st, 1e-3, which)
    _, b_off, _ = orc.assemble(prob, st, 1e-3, which)
    return (b_off - b_on), dims            # = the eps_f-scaled convection term rho div(u u/eps)


def test_convection_linear_stream(orc):
    """u(x) = U0 + G x on the x faces, v = 0, eps = 1: first-order upwind of
    d(u^2)/dx on the face-centred volume is exactly rho (2 G u_f - G^2 dx / 2)
    (fluxes at the cell centres carry the mean of the two faces, upwinded
    values from the face behind), i.e. first order in dx."""
    nx, ny, nz = 12, 3, 1
    prob = orc.Problem(nx=nx, ny=ny, nz=nz, kc=0.0)
    st = _flat_state(orc, prob)
    U0, G = 2e-4, 15.0
    xf = np.arange(nx + 1) * prob.dx
    st.ux[:] = U0 + G * xf
    C, dims = _conv_rhs_difference(orc, prob, st, 0)
    C = C.reshape(prob.face_shape(0))
    uf = U0 + G * xf[1:nx]
    np.testing.assert_allclose(C[:, :, 1:nx], np.broadcast_to(prob.rho * (2 * G * uf - G * G * prob.dx / 2),
                                                              C[:, :, 1:nx].shape), rtol=1e-12)
    assert np.all(C[:, :, [0, nx]] == 0.0)          # inlet and outlet faces carry none


def test_convection_transverse_upwinding(orc):
    """u = f(y) with v = V on every interior y face (walls v = 0): on the x
    faces the convection is rho V (f_j - f_(j-1)) / dx in the interior rows
    (the value from the face below enters), rho V f_0 / dx in the bottom row
    and -rho V f_(ny-2) / dx in the top row (no transport through the walls).
    Likewise v = g(x), u = U: on the y faces rho U (g_i - g_(i-1)) / dx, and
    rho U g_0 / dx next to the inlet, where no tangential momentum enters."""
    nx, ny = 6, 6
    prob = orc.Problem(nx=nx, ny=ny, kc=0.0)
    st = _flat_state(orc, prob)
    V = 3e-4
    yc = (np.arange(ny) + 0.5) * prob.dx
    f = 1e-4 + 2e6 * yc ** 2
    st.ux[:] = f[None, :, None]
    st.uy[:] = V
    st.uy[:, [0, ny], :] = 0.0
    C, _ = _conv_rhs_difference(orc, prob, st, 0)
    C = C.reshape(prob.face_shape(0))[0, :, 1:nx]
    r = prob.rho / prob.dx
    exp = np.empty(ny)
    exp[1:ny - 1] = r * V * (f[1:ny - 1] - f[0:ny - 2])
    exp[0] = r * V * f[0]
    exp[ny - 1] = -r * V * f[ny - 2]
    np.testing.assert_allclose(C, np.broadcast_to(exp[:, None], C.shape), rtol=1e-12, atol=1e-12 * np.abs(exp).max())
    # the y-momentum: v = g(x), u = U everywhere (inlet face included)
    st2 = _flat_state(orc, prob)
    Ux = 2e-4
    xc = (np.arange(nx) + 0.5) * prob.dx
    g = 1e-4 + 1e6 * xc ** 2
    st2.ux[:] = Ux
    st2.uy[:] = g[None, None, :]
    st2.uy[:, [0, ny], :] = 0.0
    C2, _ = _conv_rhs_difference(orc, prob, st2, 1)
    C2 = C2.reshape(prob.face_shape(1))[0, 2:ny - 1, :]     # rows away from the walls
    exp2 = np.empty(nx)
    exp2[1:] = r * Ux * (g[1:] - g[:-1])
    exp2[0] = r * Ux * g[0]
    np.testing.assert_allclose(C2, np.broadcast_to(exp2[None, :], C2.shape), rtol=1e-12)


def test_convection_vanishes_for_plug_flow(orc):
    """A uniform plug u = U (eps = 1, 3-D) carries no net momentum flux: the
    term is exactly zero on every face."""
    prob = orc.Problem(nx=10, ny=4, nz=3, kc=0.0)
    st = _flat_state(orc, prob)
    st.ux[:] = 3e-4
    C, _ = _conv_rhs_difference(orc, prob, st, 0)
    assert np.all(C == 0.0)


# ------------------------------------------------------ SIMPLE (App. A-B)

def _simple(prob, **kw):
    kw.setdefault("outer_max", 400)
    kw.setdefault("outer_tol", 1e-11)
    return dataclasses.replace(prob, simple=1, **kw)


def test_simple_loop_reaches_the_steady_poiseuille_solution(orc):
    """The quasi-static SIMPLE loop (steady momentum, relaxation 0.3, Appendix
    B) converges within one time step to the steady discrete solution: the
    plane Poiseuille profile to second order, and the same flow the one-pass
    scheme reaches after many steps."""
    ny, H = 12, 60e-6
    nx = 4 * ny
    dx = H / ny
    base = orc.Problem(nx=nx, ny=ny, dx=dx, kc=0.0, u_in=1e-4, rtol_u=1e-13, rtol_p=1e-13, rtol_c=1e-12)
    st = _flat_state(orc, base)
    d = orc.step(_simple(base, outer_max=1000, outer_tol=1e-10), st, 1.0)
    assert d["outer_its"] < 1000 and d["outer_res"] <= 1e-10
    y = (np.arange(ny) + 0.5) * dx
    exact = 6 * base.u_in * (y / H) * (1 - y / H)
    prof = st.ux[0, :, nx // 2]
    assert np.abs(prof - exact).max() / exact.max() < 1e-2
    # one-pass scheme to its steady state
    st2 = _flat_state(orc, base)
    dt = H * H * base.rho / base.mu / 50
    for _ in range(2000):
        u0 = st2.ux.copy()
        orc.step(base, st2, dt)
        if np.abs(st2.ux - u0).max() < 1e-13 * np.abs(st2.ux).max():
            break
    assert np.abs(st.ux - st2.ux).max() <= 1e-8 * np.abs(st2.ux).max()


def test_simple_fixed_point_is_independent_of_relaxation(orc):
    """Relaxation factors change the path, not the converged step: with the
    factors 0.3 and 0.7 the loop ends at the same u, p, c, and that c
    satisfies the full van Leer transport scheme (the deferred correction at
    its fixed point)."""
    from paper_2204_07019_amd import inputs
    es = inputs.rsa_discs(24, 12, seed=4, rmin=2, rmax=4, porosity=0.75)
    # Vm = 0 keeps eps at eps^n after the step, so the state holds the transport's eps
    base = orc.Problem(nx=24, ny=12, kc=1e-4, Vm=0.0, rtol_u=1e-13, rtol_p=1e-13, rtol_c=1e-13)
    out = []
    for r in (0.3, 0.7):
        st = orc.initial_state(base, es)
        p = _simple(base, relax_u=r, relax_p=r, relax_c=r, outer_tol=1e-10, outer_max=6000)
        d = orc.step(p, st, 1e-3)
        assert d["outer_res"] <= 1e-10, d["outer_res"]
        out.append((st, d))
    (a, da), (b, db) = out
    assert db["outer_its"] < da["outer_its"]
    for k in ("ux", "uy", "p", "c"):
        x, y = getattr(a, k), getattr(b, k)
        live = a.eps > 2 * base.eps_min if k in ("p", "c") else np.ones(x.shape, dtype=bool)
        assert np.abs(x - y)[live].max() <= 1e-7 * np.abs(y).max(), k
    # a's c solves the van Leer system with the correction evaluated at itself
    st = copy.deepcopy(a)
    sten, rhs, dims = orc.assemble(base, st, 1e-3, 4)
    A = orc.stencil_to_dense(sten, dims)
    r = (A @ st.c.ravel() - rhs) / sten[0]
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(rhs / sten[0])


def test_simple_adaptive_time_step(orc):
    """Quasi-static stepping with Appendix D's bound: the flow and transport
    do not depend on dt, the solid step is deps_max / max |V_m Rbar| (a cap
    of dt = 1e9 s never binds) and the largest change of eps is deps_max."""
    from paper_2204_07019_amd import inputs
    es = inputs.calcite_post(48, 24, 14, 12, 5)
    base = orc.Problem(nx=48, ny=24, kc=1e-4, rtol_u=1e-12, rtol_p=1e-12, rtol_c=1e-12)
    p = _simple(base, deps_max=0.005, outer_tol=1e-10)
    st = orc.initial_state(base, es)
    d1 = orc.step(p, st, 1e9)
    st2 = orc.initial_state(base, es)
    d2 = orc.step(p, st2, 1e6)
    assert d1["dt_solid"] < 1e6
    assert d1["dt_solid"] == pytest.approx(d2["dt_solid"], rel=1e-9)
    assert d1["max_deps"] == pytest.approx(0.005, rel=1e-12)
    np.testing.assert_allclose(st.c, st2.c, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------- transient (Sec. 2.2)

def test_transient_diffusion_erfc_first_order_in_time(orc):
    """With the storage term on, diffusion from the inlet (c_in, no flow, no
    solid) into a long fluid column follows c = c_in erfc(x / 2 sqrt(D t));
    backward Euler makes the error first order in dt."""
    from scipy.special import erfc
    D, T, nx, dx = 1e-9, 0.05, 200, 1e-6
    errs = []
    for nsteps in (10, 20, 40):
        prob = orc.Problem(nx=nx, ny=1, dx=dx, D=D, kc=0.0, u_in=0.0, c_in=1.0, transient=1,
                           rtol_u=1e-13, rtol_p=1e-13, rtol_c=1e-13)
        st = _flat_state(orc, prob)
        dt = T / nsteps
        for _ in range(nsteps):
            d = orc.step(prob, st, dt)
            assert abs(d["acid_balance_rel"]) < 1e-10
        x = (np.arange(nx) + 0.5) * dx
        exact = erfc(x / (2 * math.sqrt(D * T)))
        errs.append(np.abs(st.c[0, 0] - exact).max())
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4, errs


def test_transient_balances_and_continuity_source(orc):
    """With storage and the dissolution source of Eq. contDBS on, the acid
    balance in - out - consumed - storage closes to the solver tolerance and
    the net outflow of fluid volume equals the summed source
    Rbar M_ws (1/rho_s - 1/rho) V of the lagged rates."""
    from paper_2204_07019_amd import inputs
    es = inputs.calcite_post(40, 20, 12, 10, 4)
    prob = orc.Problem(nx=40, ny=20, kc=1e-4, transient=1, Vm_f=1e-4, rtol_u=1e-13, rtol_p=1e-13,
                       rtol_c=1e-14)
    st = orc.initial_state(prob, es)
    st.c[:] = prob.c_in          # acid everywhere already: the solid reacts from the first step
    S = prob.dx ** 2
    for k in range(4):
        d = orc.step(prob, st, 1e-3)
        assert abs(d["acid_balance_rel"]) < 1e-10, d
        assert abs(d["solid_balance_rel"]) < 1e-10
        q_out = S * st.ux[:, :, -1].sum()
        q_in = S * st.ux[:, :, 0].sum()
        if k == 0:
            assert d["div_source"] == 0.0           # no earlier rate: no source yet
        else:
            assert d["div_source"] < 0.0            # Vm < Vm_f: dissolution shrinks the fluid volume
        assert abs((q_out - q_in) - d["div_source"]) <= 1e-9 * abs(q_in)
    assert d["acid_accum"] != 0.0


# ----------------------------------------------- VoS-psi variants (Sec. 2.4)

@pytest.mark.parametrize("nz", [1, 5])
def test_isolated_remnant_psi_variants(orc, nz):
    """One partially dissolved cell in fluid, uniform c.  Centred gradient with
    psi = 1: the remnant's own gradient vanishes and its 2 n_d neighbours carry
    |g| = (1 - eps_P)/(2 dx): total rate n_d k_c c (1 - eps_P) dx^2 (= iVoS's),
    none of it in the remnant.  Decentred gradient with psi = 1: every one-sided
    difference toward the fluid is (1 - eps_P)/dx, so the remnant carries
    |g| = sqrt(n_d)(1 - eps_P)/dx and its neighbours none: it dissolves."""
    n, ep, cc = 5, 0.35, 2.0
    nd = 2 if nz == 1 else 3
    k0 = nz // 2
    for scheme in (0, 1):
        prob = orc.Problem(nx=n, ny=n, nz=nz, kc=3e-4, model=1, psi_kind=1, grad_scheme=scheme)
        eps = np.ones(prob.cell_shape)
        eps[k0, 2, 2] = ep
        c = np.full(prob.cell_shape, cc)
        rbar, _, g, _, _ = orc.reaction(prob, 1e-3, eps, c)
        V = prob.dx ** 3
        if scheme == 0:
            assert rbar[k0, 2, 2] == 0.0
            assert (rbar * V).sum() == pytest.approx(nd * prob.kc * cc * (1 - ep) * prob.dx ** 2, rel=1e-13)
        else:
            assert rbar[k0, 2, 2] == pytest.approx(prob.kc * cc * math.sqrt(nd) * (1 - ep) / prob.dx, rel=1e-13)
            other = rbar.copy()
            other[k0, 2, 2] = 0.0
            assert np.all(other == 0.0)


def test_plane_front_decentred_area_in_the_solid_cell(orc):
    """Flat front, decentred gradient and psi = 1: the whole interface area
    A (1 - eps_min) sits in the first solid cell, so with frozen uniform c the
    total rate is k_c c A (1 - eps_min), as for iVoS, all of it dissolving
    that cell."""
    m, nx, ny = 6, 16, 4
    prob = orc.Problem(nx=nx, ny=ny, model=1, psi_kind=1, grad_scheme=1, kc=2e-4)
    es = np.zeros((1, ny, nx))
    es[:, :, m:] = 1.0
    eps = orc.eps_from_solid(prob, es)
    c = np.full(prob.cell_shape, 3.0)
    rbar, _, g, _, _ = orc.reaction(prob, 1e-3, eps, c)
    A = ny * prob.dx ** 2
    V = prob.dx ** 3
    assert (rbar * V).sum() == pytest.approx(prob.kc * 3.0 * A * (1 - prob.eps_min), rel=1e-13)
    mask = np.zeros_like(rbar, dtype=bool)
    mask[:, :, m] = True
    assert np.all(rbar[~mask] == 0.0)


def test_variant_combinations_rejected(orc):
    """The decentred gradient is a VoS-psi variant (iVoS keeps its central
    normals); lambda of VoS-psi' is fitted to eps (1 - eps), not to psi = 1."""
    st = None
    for kw in (dict(model=0, grad_scheme=1), dict(model=2, psi_kind=1), dict(drive=2),
               dict(simple=1, relax_u=0.0), dict(simple=1, outer_max=0)):
        prob = orc.Problem(nx=6, ny=4, **kw)
        st = orc.initial_state(prob, np.zeros(prob.cell_shape))
        d = orc.step(prob, st, 1e-3, check=False)
        assert d["status"] == 1, kw


# --------------------------------------------------------- diagnostics

def test_r_omega_and_darcy_velocity_diagnostics(orc):
    """R_Omega of Section 3.3 is the porosity change per V_m dt_s: by the solid
    balance of Eq. mbs it equals (dt_s V_m sum Rbar V - clipped volume) /
    (V_total V_m dt_s), two outputs computed apart (the porosity change and
    the rates); U_D is u_in under the velocity drive."""
    from paper_2204_07019_amd import inputs
    es = inputs.calcite_post(40, 20, 12, 10, 4)
    prob = orc.Problem(nx=40, ny=20, kc=1e-4, rtol_u=1e-13, rtol_p=1e-13, rtol_c=1e-13)
    st = orc.initial_state(prob, es)
    for _ in range(3):
        d = orc.step(prob, st, 1e-3)
    vtot = prob.nx * prob.ny * prob.dx ** 3
    dts = d["dt_solid"]
    expect = (dts * prob.Vm * d["solid_rate"] - d["clipped_volume"]) / (vtot * prob.Vm * dts)
    assert d["R_omega"] == pytest.approx(expect, rel=1e-9)
    assert d["R_omega"] > 0
    assert d["U_D"] == pytest.approx(prob.u_in, rel=1e-14)


def test_solid_step_bound_ignores_cells_held_by_the_clip(orc):
    """Appendix D bounds the actual change of eps.  With the transported field
    zero and a random lagged field, iVoS rates are eps_P times the divergence
    of the van Leer corrections alone, largest in fluid cells (eps = 1) where a
    positive rate is held by the clip.  When such a cell carries the largest
    |rate|, the step must still reach deps_max in some free cell (a bound
    taken over the held cells too would stop short of it)."""
    from paper_2204_07019_amd import inputs
    es = inputs.calcite_post(24, 16, 12, 8, 4)
    prob = orc.Problem(nx=24, ny=16, kc=2e-4)
    eps0 = orc.eps_from_solid(prob, es)
    found = 0
    for seed in range(6):
        rng = np.random.default_rng(seed)
        eps = np.where((eps0 > prob.eps_min) & (eps0 < 1.0), rng.uniform(0.2, 0.8, eps0.shape), eps0)
        c_new = np.zeros(eps.shape)
        c_old = rng.uniform(0.0, 10.0, eps.shape)
        rbar, *_ = orc.reaction(prob, 1e-3, eps, c_new, c_old)
        rate = prob.Vm * rbar
        i = np.argmax(np.abs(rate))
        if not (rate.ravel()[i] > 0 and eps.ravel()[i] == 1.0):
            continue
        found += 1
        lim = 0.2 * np.abs(rate).max() * 1e-3
        lp = dataclasses.replace(prob, deps_max=lim)
        _, _, _, _, e1, dts = orc.reaction(lp, 1e-3, eps, c_new, c_old, return_dt=True)
        change = np.abs(e1 - eps)
        assert change.max() == pytest.approx(lim, rel=1e-9)
        assert dts < 1e-3 and change.ravel()[i] == 0.0
    assert found >= 3


def test_step_is_insensitive_to_rounding_of_eps(orc):
    """The interface normal -grad eps / |grad eps| (Section 2.3) is undefined
    where eps is flat; it is taken as 0 where eps varies by at most 1e-6 across
    a cell.  With that reading a relative perturbation of eps at the rounding
    level (1e-15) changes nothing measurable over 8 dissolving post steps:
    the concentration by < 1e-10, the change of eps by < 1e-8.  (A threshold
    at 1e-10 / dx let unit reactive fluxes follow rounding-level gradients and
    amplified the same perturbation to ~2e-6 in c.)"""
    from paper_2204_07019_amd import inputs
    es, prm = inputs.workload("post")
    nz, ny, nx = es.shape
    keys = ("mu", "rho", "D", "k0", "kc", "Vm", "zeta", "c_in", "eps_min", "u_in", "p_out")
    prob = orc.Problem(nx=nx, ny=ny, nz=nz, dx=prm["dx"], **{k: prm[k] for k in keys},
                       rtol_u=1e-12, rtol_p=1e-12, rtol_c=1e-12)
    st = orc.initial_state(prob, es)
    for _ in range(12):
        orc.step(prob, st, 1e-3)
    rng = np.random.default_rng(0)
    a, b = st.copy(), st.copy()
    b.eps = np.minimum(b.eps * (1 + 1e-15 * rng.standard_normal(b.eps.shape)), 1.0)
    for _ in range(8):
        orc.step(prob, a, 1e-3)
        orc.step(prob, b, 1e-3)
    rel = lambda x, y: np.linalg.norm(x - y) / np.linalg.norm(y)
    assert rel(b.c, a.c) < 1e-10
    assert rel(b.eps - st.eps, a.eps - st.eps) < 1e-8

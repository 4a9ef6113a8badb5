"""FP64 CPU oracle of one Volume-of-Solid step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it, and
it shares no code with the HIP path: ``vos_oracle.c`` is a separate, plain C
implementation written from the paper (Maes, Soulaine & Menke), built with gcc.

Every routine here is marshalling around ``vos_oracle.c``; the arithmetic lives
there, each part citing the section / equation it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vos_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")

MODEL_IVOS, MODEL_PSI, MODEL_PSI_PRIME = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Prob(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("mu", C.c_double), ("rho", C.c_double), ("D", C.c_double), ("k0", C.c_double),
                ("kc", C.c_double), ("Vm", C.c_double), ("zeta", C.c_double), ("c_in", C.c_double),
                ("eps_min", C.c_double), ("u_in", C.c_double), ("p_out", C.c_double),
                ("model", C.c_int),
                ("rtol_u", C.c_double), ("rtol_p", C.c_double), ("rtol_c", C.c_double),
                ("maxit_u", C.c_int), ("maxit_p", C.c_int), ("maxit_c", C.c_int),
                ("deps_max", C.c_double),
                ("drive", C.c_int), ("p_in", C.c_double), ("convection", C.c_int),
                ("grad_scheme", C.c_int), ("psi_kind", C.c_int), ("transient", C.c_int),
                ("Vm_f", C.c_double), ("simple", C.c_int), ("outer_max", C.c_int),
                ("outer_tol", C.c_double), ("relax_u", C.c_double), ("relax_p", C.c_double),
                ("relax_c", C.c_double), ("solid_dt", C.c_double)]


class _Diag(C.Structure):
    _fields_ = [("it_u", C.c_int * 3), ("it_p", C.c_int), ("it_c", C.c_int),
                ("res_u", C.c_double * 3), ("res_p", C.c_double), ("res_c", C.c_double),
                ("lam", C.c_double), ("solid_volume", C.c_double), ("surface_area", C.c_double),
                ("porosity", C.c_double), ("dP", C.c_double), ("K", C.c_double),
                ("acid_in", C.c_double), ("acid_out", C.c_double), ("acid_consumed", C.c_double),
                ("solid_rate", C.c_double), ("acid_balance_rel", C.c_double),
                ("solid_balance_rel", C.c_double), ("clipped_volume", C.c_double),
                ("max_deps", C.c_double), ("alpha", C.c_double), ("dt_solid", C.c_double),
                ("U_D", C.c_double), ("R_omega", C.c_double), ("acid_accum", C.c_double),
                ("outer_its", C.c_int), ("outer_res", C.c_double), ("div_source", C.c_double)]


class _Aux(C.Structure):
    _fields_ = [("eps_prev", C.POINTER(C.c_double)), ("rbar_prev", C.POINTER(C.c_double))]


class _Out(C.Structure):
    _fields_ = [("ustar", C.POINTER(C.c_double) * 3), ("rbar", C.POINTER(C.c_double)),
                ("sink", C.POINTER(C.c_double)), ("gmag", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_step.argtypes = [C.POINTER(_Prob), C.c_double, dp, dp, dp, dp, dp, dp,
                               C.POINTER(_Aux), C.POINTER(_Out), C.POINTER(_Diag)]
        L.orc_step.restype = C.c_int
        L.orc_eps_from_solid.argtypes = [C.POINTER(_Prob), dp, dp]
        L.orc_assemble.argtypes = [C.POINTER(_Prob), C.c_double, dp, dp, dp, dp, dp, dp,
                                   C.POINTER(_Aux), C.c_int, dp, dp]
        L.orc_assemble.restype = C.c_int
        L.orc_solve_stencil.argtypes = [C.POINTER(C.c_int), dp, dp, dp, C.c_int, C.c_double,
                                        C.c_int, C.POINTER(C.c_int), dp]
        L.orc_solve_stencil.restype = C.c_int
        L.orc_reaction.argtypes = [C.POINTER(_Prob), C.c_double, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_reaction.restype = C.c_int
        L.orc_vanleer_face.argtypes = [C.c_double] * 3
        L.orc_vanleer_face.restype = C.c_double
        L.orc_r_omega.argtypes = [C.c_double] * 4
        L.orc_r_omega.restype = C.c_double
        _lib = L
    return _lib


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int = 1
    dx: float = 5e-6
    mu: float = 1e-3
    rho: float = 1000.0
    D: float = 1e-9
    k0: float = 1e-15
    kc: float = 1e-4
    Vm: float = 3.69e-5
    zeta: float = 1.0
    c_in: float = 10.0
    eps_min: float = 1e-4
    u_in: float = 1e-4
    p_out: float = 0.0
    model: int = MODEL_IVOS
    rtol_u: float = 1e-12
    rtol_p: float = 1e-12
    rtol_c: float = 1e-12
    maxit_u: int = 200000
    maxit_p: int = 200000
    maxit_c: int = 200000
    deps_max: float = 0.0   # > 0: largest change of eps per step (Appendix D), by a shorter solid step
    drive: int = 0          # 0: inlet plug velocity u_in; 1: inlet pressure p_in
    p_in: float = 0.0
    convection: int = 0     # 1: explicit first-order upwind momentum convection (Eq. momentumDBS)
    grad_scheme: int = 0    # 0: central gradient of eps; 1: decentred (VoS-psi variants only)
    psi_kind: int = 0       # 0: psi = lambda eps (1 - eps); 1: psi = 1
    transient: int = 0      # 1: storage d(eps c)/dt and the continuity source of Eq. contDBS
    Vm_f: float = 1e-4      # M_ws / rho of the fluid [m3/mol] (calcite 0.1 kg/mol in water)
    simple: int = 0         # 1: quasi-static SIMPLE outer loop (Appendices A, B)
    outer_max: int = 50
    outer_tol: float = 1e-8
    relax_u: float = 0.3
    relax_p: float = 0.3
    relax_c: float = 1.0
    solid_dt: float = 0.0   # > 0: the solid update's own step; dt is then the flow's pseudo time step

    def c_struct(self) -> _Prob:
        return _Prob(**asdict(self))

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def face_shape(self, d: int):
        """(nz, ny, nx)-ordered shape of the face grid of direction d."""
        n = [self.nx, self.ny, self.nz]
        n[d] += 1
        return (n[2], n[1], n[0])

    @property
    def cell_shape(self):
        return (self.nz, self.ny, self.nx)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class State:
    eps: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    p: np.ndarray
    c: np.ndarray
    # carried for the transient terms: eps at the previous step's start and the
    # previous step's reaction rate (None: eps and zeros)
    eps_prev: np.ndarray = None
    rbar_prev: np.ndarray = None

    def __post_init__(self):
        if self.eps_prev is None:
            self.eps_prev = np.array(self.eps, dtype=np.float64, copy=True)
        if self.rbar_prev is None:
            self.rbar_prev = np.zeros_like(self.eps, dtype=np.float64)

    def copy(self) -> "State":
        return State(*(np.array(getattr(self, k), dtype=np.float64, copy=True)
                       for k in ("eps", "ux", "uy", "uz", "p", "c", "eps_prev", "rbar_prev")))

    def aux(self) -> "_Aux":
        return _Aux(_ptr(self.eps_prev), _ptr(self.rbar_prev))


def eps_from_solid(prob: Problem, eps_s: np.ndarray) -> np.ndarray:
    """eps = clamp(1 - eps_s, eps_min, 1) (Appendix C: eps_f = 1e-4 in the solid)."""
    es = np.ascontiguousarray(eps_s, dtype=np.float64).reshape(prob.cell_shape)
    out = np.empty_like(es)
    pr = prob.c_struct()
    lib().orc_eps_from_solid(C.byref(pr), _ptr(es), _ptr(out))
    return out


def initial_state(prob: Problem, eps_s: np.ndarray) -> State:
    """Fluid at rest, p = p_out, c = 0 (a seeded start both paths share); the
    inlet faces carry u_in under the velocity drive, 0 under the pressure drive."""
    eps = eps_from_solid(prob, eps_s)
    ux = np.zeros(prob.face_shape(0))
    ux[:, :, 0] = prob.u_in if prob.drive == 0 else 0.0
    return State(eps=eps, ux=ux, uy=np.zeros(prob.face_shape(1)), uz=np.zeros(prob.face_shape(2)),
                 p=np.full(prob.cell_shape, prob.p_out), c=np.zeros(prob.cell_shape))


def step(prob: Problem, st: State, dt: float, intermediates: bool = False, check: bool = True):
    """Advance ``st`` in place by one step; return the diagnostics dict
    (and the intermediates when asked)."""
    pr = prob.c_struct()
    dg = _Diag()
    out = _Out()
    inter = {}
    if intermediates:
        inter = {"ustar_x": np.zeros(prob.face_shape(0)), "ustar_y": np.zeros(prob.face_shape(1)),
                 "ustar_z": np.zeros(prob.face_shape(2)), "rbar": np.zeros(prob.cell_shape),
                 "sink": np.zeros(prob.cell_shape), "gmag": np.zeros(prob.cell_shape)}
        out.ustar[0] = _ptr(inter["ustar_x"])
        out.ustar[1] = _ptr(inter["ustar_y"])
        out.ustar[2] = _ptr(inter["ustar_z"])
        out.rbar = _ptr(inter["rbar"])
        out.sink = _ptr(inter["sink"])
        out.gmag = _ptr(inter["gmag"])
    ax = st.aux()
    rc = lib().orc_step(C.byref(pr), dt, _ptr(st.eps), _ptr(st.ux), _ptr(st.uy), _ptr(st.uz),
                        _ptr(st.p), _ptr(st.c), C.byref(ax), C.byref(out), C.byref(dg))
    d = {k: (list(getattr(dg, k)) if k in ("it_u", "res_u") else getattr(dg, k))
         for k, _ in _Diag._fields_}
    d["lambda"] = d.pop("lam")
    d["status"] = rc
    if check and rc != 0:
        raise RuntimeError(f"oracle step failed with status {rc}: {d}")
    return (d, inter) if intermediates else d


def assemble(prob: Problem, st: State, dt: float, which: int):
    """The stencil (7, N) and right-hand side of one of the step's systems.
    which: 0/1/2 momentum x/y/z (from u^n, p^n), 3 pressure (st.u* as u,
    p^n), 4 transport (corrected u, c^n; rows unscaled)."""
    n = [prob.nx, prob.ny, prob.nz]
    if which < 3:
        n[which] += 1
    N = n[0] * n[1] * n[2]
    sten = np.zeros((7, N))
    rhs = np.zeros(N)
    pr = prob.c_struct()
    ax = st.aux()
    rc = lib().orc_assemble(C.byref(pr), dt, _ptr(st.eps), _ptr(st.ux), _ptr(st.uy), _ptr(st.uz),
                            _ptr(st.p), _ptr(st.c), C.byref(ax), which, _ptr(sten), _ptr(rhs))
    if rc:
        raise RuntimeError(f"orc_assemble failed ({rc})")
    return sten, rhs, tuple(n)


def stencil_to_dense(sten: np.ndarray, dims) -> np.ndarray:
    """Dense matrix of a 7-point stencil over a grid of dims (nx, ny, nz)."""
    nx, ny, nz = dims
    N = nx * ny * nz
    A = np.zeros((N, N))
    idx = np.arange(N)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    A[idx, idx] = sten[0]
    for slot, (off, ok) in enumerate([(-1, i > 0), (1, i < nx - 1), (-nx, j > 0), (nx, j < ny - 1),
                                      (-nx * ny, k > 0), (nx * ny, k < nz - 1)], start=1):
        r = idx[ok]
        A[r, r + off] = sten[slot][ok]
    return A


def solve_stencil(sten: np.ndarray, dims, b: np.ndarray, x0=None, kind: int = 0,
                  rtol: float = 1e-12, maxit: int = 100000):
    """Run the oracle's own Jacobi-PCG (kind 0) or row-scaled BiCGStab (kind 1)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    n = (C.c_int * 3)(*dims)
    its = C.c_int()
    rr = C.c_double()
    s = np.ascontiguousarray(sten, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    rc = lib().orc_solve_stencil(n, _ptr(s), _ptr(bb), _ptr(x), kind, rtol, maxit,
                                 C.byref(its), C.byref(rr))
    return x, rc, its.value, rr.value


def reaction(prob: Problem, dt: float, eps: np.ndarray, c_new: np.ndarray, c_old=None,
             return_dt: bool = False):
    """S1 + S6 + the solid update with a prescribed concentration: returns
    (Rbar, sink, gmag, lambda, eps_new), plus the solid step taken when
    return_dt (dt, or shorter under prob.deps_max)."""
    e = np.array(eps, dtype=np.float64, copy=True).reshape(prob.cell_shape)
    cn = np.ascontiguousarray(c_new, dtype=np.float64).reshape(prob.cell_shape)
    co = cn if c_old is None else np.ascontiguousarray(c_old, dtype=np.float64).reshape(prob.cell_shape)
    rbar = np.zeros(prob.cell_shape)
    sink = np.zeros(prob.cell_shape)
    gmag = np.zeros(prob.cell_shape)
    lam = C.c_double()
    dts = C.c_double()
    pr = prob.c_struct()
    rc = lib().orc_reaction(C.byref(pr), dt, _ptr(e), _ptr(cn), _ptr(co), _ptr(rbar), _ptr(sink),
                            _ptr(gmag), C.byref(lam), C.byref(dts))
    if rc:
        raise RuntimeError(f"orc_reaction failed ({rc})")
    if return_dt:
        return rbar, sink, gmag, lam.value, e, dts.value
    return rbar, sink, gmag, lam.value, e


def vanleer_face(phi_u: float, phi_c: float, phi_d: float) -> float:
    return lib().orc_vanleer_face(phi_u, phi_c, phi_d)


def r_omega(rho_s: float, M_w: float, dphi: float, dt: float) -> float:
    return lib().orc_r_omega(rho_s, M_w, dphi, dt)

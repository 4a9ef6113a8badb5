"""Thin ctypes binding of libvos.so (include/vos.h): argument marshalling only.

Every step of the method runs in the gfx950 kernels of libvos.so.  PyTorch is
used for device memory (the workspace and field buffers) and the stream.  If
the library is missing the import of this module fails loudly: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, asdict, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libvos.so")

VOS_OK, VOS_ERR_ARG, VOS_ERR_DEVICE, VOS_ERR_NOCONV, VOS_ERR_OOM, VOS_ERR_STATE = range(6)
IVOS, PSI, PSI_PRIME = 0, 1, 2
FP64, MIXED = 0, 1
FREEZE_SOLID = 1
KERNELS = {"v_restrict": 0, "v_post": 1, "v_pre": 2, "v_coarse": 3, "p_apply": 4, "adr_apply": 5,
           "v_down": 6, "v_up": 7, "p_pre3d": 8, "p_sweep3d": 9, "p_restrict3d": 10, "p_post3d": 11,
           "c_pre3d": 12, "c_sweep3d": 13, "c_restrict3d": 14, "c_post3d": 15, "c_down3d": 16, "c_up3d": 17,
           "m_down3d": 18, "m_up3d": 19}
FIELDS = {"eps": 0, "ux": 1, "uy": 2, "uz": 3, "p": 4, "c": 5, "ustar_x": 6, "ustar_y": 7,
          "ustar_z": 8, "rbar": 9, "gmag": 10, "pdiag": 11}


class VosError(RuntimeError):
    def __init__(self, status: int, msg: str, diag: Optional[dict] = None):
        super().__init__(f"vos status {status}: {msg}")
        self.status = status
        self.diag = diag


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("mu", C.c_double), ("rho", C.c_double), ("D", C.c_double), ("k0", C.c_double),
                ("kc", C.c_double), ("Vm", C.c_double), ("zeta", C.c_double), ("c_in", C.c_double),
                ("eps_min", C.c_double), ("u_in", C.c_double), ("p_out", C.c_double),
                ("model", C.c_int), ("drive", C.c_int), ("p_in", C.c_double), ("convection", C.c_int),
                ("grad_scheme", C.c_int), ("psi_kind", C.c_int), ("transient", C.c_int),
                ("Vm_f", C.c_double)]


# vos_params fields a params dict may leave out (the single-pass step's settings)
PARAM_DEFAULTS = {"drive": 0, "p_in": 0.0, "convection": 0, "grad_scheme": 0, "psi_kind": 0,
                  "transient": 0, "Vm_f": 1e-4}


def make_params(params: dict) -> "_Params":
    """vos_params from a dict of its fields (the optional ones default)."""
    keys = [k for k, _ in _Params._fields_]
    return _Params(**{k: params[k] if k in params else PARAM_DEFAULTS[k] for k in keys})


class _Opts(C.Structure):
    _fields_ = [("rtol_u", C.c_double), ("rtol_p", C.c_double), ("rtol_c", C.c_double),
                ("maxit_u", C.c_int), ("maxit_p", C.c_int), ("maxit_c", C.c_int),
                ("precision", C.c_int), ("mg_nu", C.c_int), ("check_every", C.c_int),
                ("use_graphs", C.c_int), ("coarse_cells", C.c_int), ("level_kernels", C.c_int),
                ("p_fp32_its", C.c_int), ("extrapolate", C.c_int), ("setup_every", C.c_int),
                ("deps_max", C.c_double), ("simple", C.c_int), ("outer_max", C.c_int),
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
                ("max_deps", C.c_double), ("alpha", C.c_double), ("t_ms", C.c_double * 6),
                ("guess", C.c_int), ("res0_prev", C.c_double), ("res0_guess", C.c_double),
                ("guess_error_drop", C.c_double), ("it_p_fp64", C.c_int), ("dt_solid", C.c_double),
                ("U_D", C.c_double), ("R_omega", C.c_double), ("acid_accum", C.c_double),
                ("outer_its", C.c_int), ("outer_res", C.c_double), ("div_source", C.c_double)]


_lib = None


def lib():
    """Load libvos.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2204_07019_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.vos_workspace_bytes.argtypes = [C.POINTER(_Grid), C.POINTER(_Opts), C.POINTER(C.c_size_t)]
        L.vos_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Opts), vp, C.c_size_t,
                                 vp, C.POINTER(vp)]
        L.vos_destroy.argtypes = [vp]
        L.vos_set_solid_fraction.argtypes = [vp, vp, C.c_int]
        L.vos_set_field.argtypes = [vp, C.c_int, vp, C.c_int]
        L.vos_set_params.argtypes = [vp, C.POINTER(_Params)]
        L.vos_get_field.argtypes = [vp, C.c_int, vp, C.c_int]
        L.vos_field_ptr.argtypes = [vp, C.c_int, C.POINTER(vp)]
        L.vos_step.argtypes = [vp, C.c_double, C.c_int, C.c_int, C.POINTER(_Diag)]
        L.vos_diagnostics.argtypes = [vp, C.POINTER(_Diag)]
        L.vos_time_kernel.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.vos_solve_pressure.argtypes = [vp, C.c_double, vp, C.c_int, C.POINTER(_Diag)]
        L.vos_initialize.argtypes = [vp, C.c_double, C.c_int, C.c_double, C.POINTER(_Diag)]
        L.vos_state_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.vos_get_state.argtypes = [vp, vp, C.c_size_t]
        L.vos_set_state.argtypes = [vp, vp, C.c_size_t]
        L.vos_solve_pressure_noalloc.argtypes = [C.POINTER(_Grid), C.POINTER(_Params), C.POINTER(_Opts), C.c_double,
                                                 vp, vp, vp, vp, vp, vp, C.POINTER(_Diag)]
        L.vos_solve_pressure_noalloc.restype = C.c_int
        L.vos_last_error.restype = C.c_char_p
        for name in ("vos_workspace_bytes", "vos_create", "vos_destroy", "vos_set_solid_fraction",
                     "vos_set_field", "vos_set_params", "vos_get_field", "vos_field_ptr", "vos_step", "vos_diagnostics",
                     "vos_time_kernel", "vos_solve_pressure", "vos_initialize", "vos_state_bytes",
                     "vos_get_state", "vos_set_state"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, diag=None):
    if rc != VOS_OK:
        raise VosError(rc, lib().vos_last_error().decode(), diag)


def diag_to_dict(dg: _Diag) -> dict:
    d = {}
    for k, _ in _Diag._fields_:
        v = getattr(dg, k)
        d[k] = list(v) if k in ("it_u", "res_u", "t_ms") else v
    d["lambda"] = d.pop("lam")
    return d


@dataclass
class Opts:
    rtol_u: float = 1e-8
    rtol_p: float = 1e-8
    rtol_c: float = 1e-8
    maxit_u: int = 20000
    maxit_p: int = 2000
    maxit_c: int = 20000
    precision: int = FP64
    mg_nu: int = 0          # 0: library default (pressure 4 in 2-D, 3 in 3-D; momentum 2)
    check_every: int = 8
    use_graphs: int = 1
    coarse_cells: int = 0
    level_kernels: int = 0  # 0: fused fine-level multigrid kernels, 1: one plain kernel per sweep
    p_fp32_its: int = 0     # mixed: cap on FP32-preconditioned pressure iterations (0: stall detection only)
    extrapolate: int = 0    # 1: solves start from 2 x^n - x^(n-1) of the last two steps; 2: adaptive quadratic
    setup_every: int = 0    # rebuild the multigrid hierarchies every this many steps (0, 1: every step)
    deps_max: float = 0.0   # > 0: the solid update's step is cut so that no eps changes by more (Appendix D)
    simple: int = 0         # 1: quasi-static SIMPLE loop per step (Appendices A, B)
    outer_max: int = 50
    outer_tol: float = 1e-8
    relax_u: float = 0.3
    relax_p: float = 0.3
    relax_c: float = 1.0
    solid_dt: float = 0.0   # > 0: the solid update's own step; dt is then the flow's pseudo time step


class Sim:
    """One simulation on one GPU.  ``params`` holds the vos_params fields
    (mu, rho, D, k0, kc, Vm, zeta, c_in, eps_min, u_in, p_out, model)."""

    def __init__(self, nx: int, ny: int, nz: int, dx: float, params: dict,
                 opts: Optional[Opts] = None, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.grid = _Grid(nx, ny, nz, dx)
        self.params = make_params(params)
        self.opts = _Opts(**asdict(opts or Opts()))
        nbytes = C.c_size_t()
        _check(lib().vos_workspace_bytes(C.byref(self.grid), C.byref(self.opts), C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority): the legacy null stream cannot be graph-captured
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        _check(lib().vos_create(C.byref(self.grid), C.byref(self.params), C.byref(self.opts),
                                C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    @classmethod
    def borrowed(cls, handle, nx: int, ny: int, nz: int, dx: float, params: dict, device: str = "cuda:0"):
        """Wrap a handle owned elsewhere (a batch instance): same methods,
        close() does not destroy it."""
        import torch
        self = cls.__new__(cls)
        self.torch = torch
        self.device = torch.device(device)
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.grid = _Grid(nx, ny, nz, dx)
        self.params = make_params(params)
        self._h = handle
        self._borrowed = True
        return self

    def close(self):
        if getattr(self, "_borrowed", False):
            self._h = None
            return
        if getattr(self, "_h", None):
            lib().vos_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- fields
    def field_shape(self, name: str):
        nz, ny, nx = self.shape
        if name in ("ux", "ustar_x"):
            return (nz, ny, nx + 1)
        if name in ("uy", "ustar_y"):
            return (nz, ny + 1, nx)
        if name in ("uz", "ustar_z"):
            return (nz + 1, ny, nx)
        return self.shape

    def set_solid_fraction(self, eps_s):
        t = self._as_device(eps_s, self.shape)
        _check(lib().vos_set_solid_fraction(self._h, C.c_void_p(t.data_ptr()), 1))

    def set_params(self, params: dict):
        keys = [k for k, _ in _Params._fields_]
        merged = {k: params.get(k, getattr(self.params, k)) for k in keys}
        p = _Params(**merged)
        _check(lib().vos_set_params(self._h, C.byref(p)))
        self.params = p

    def set(self, name: str, arr):
        t = self._as_device(arr, self.field_shape(name))
        _check(lib().vos_set_field(self._h, FIELDS[name], C.c_void_p(t.data_ptr()), 1))

    def get(self, name: str):
        """Copy of a field as a device tensor (float64)."""
        out = self.torch.empty(self.field_shape(name), dtype=self.torch.float64, device=self.device)
        _check(lib().vos_get_field(self._h, FIELDS[name], C.c_void_p(out.data_ptr()), 1))
        return out

    def get_numpy(self, name: str) -> np.ndarray:
        return self.get(name).cpu().numpy()

    def _as_device(self, arr, shape):
        torch = self.torch
        t = torch.as_tensor(np.asarray(arr) if not isinstance(arr, torch.Tensor) else arr)
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        # the library reads it on its own stream: finish torch's copy first
        torch.cuda.current_stream(self.device).synchronize()
        if tuple(t.shape) != tuple(shape) and t.numel() != int(np.prod(shape)):
            raise ValueError(f"expected {shape}, got {tuple(t.shape)}")
        return t

    # ---------------------------------------------------------------- stepping
    def step(self, dt: float, nsteps: int = 1, freeze_solid: bool = False) -> dict:
        dg = _Diag()
        rc = lib().vos_step(self._h, dt, nsteps, FREEZE_SOLID if freeze_solid else 0, C.byref(dg))
        _check(rc, diag_to_dict(dg))
        return diag_to_dict(dg)

    def time_kernel(self, family: str, reps: int = 50) -> dict:
        """Average duration and algorithmic bytes of one launch of a kernel
        family, timed back to back on the live state with HIP events."""
        ms, by = C.c_double(), C.c_double()
        _check(lib().vos_time_kernel(self._h, KERNELS[family], reps, C.byref(ms), C.byref(by)))
        return {"avg_ms": ms.value, "bytes": by.value}

    def diagnostics(self) -> dict:
        dg = _Diag()
        _check(lib().vos_diagnostics(self._h, C.byref(dg)))
        return diag_to_dict(dg)

    def solve_pressure(self, dt: float, guess=None) -> dict:
        """The pressure equation alone from the current state (vos_solve_pressure)."""
        dg = _Diag()
        ptr = None
        if guess is not None:
            g = self._as_device(guess, self.shape)
            ptr = C.c_void_p(g.data_ptr())
        rc = lib().vos_solve_pressure(self._h, dt, ptr, 1, C.byref(dg))
        _check(rc, diag_to_dict(dg))
        return diag_to_dict(dg)

    def initialize(self, dt: float, max_iters: int = 200, tol: float = 1e-10) -> dict:
        """Steady flow with eps frozen, then c^0 (vos_initialize)."""
        dg = _Diag()
        rc = lib().vos_initialize(self._h, dt, max_iters, tol, C.byref(dg))
        _check(rc, diag_to_dict(dg))
        return diag_to_dict(dg)

    def get_state(self) -> bytes:
        """Checkpoint of the physical state (vos_get_state) as bytes."""
        n = C.c_size_t()
        _check(lib().vos_state_bytes(self._h, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check(lib().vos_get_state(self._h, buf, n.value))
        return bytes(buf)

    def set_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        _check(lib().vos_set_state(self._h, buf, len(state)))


def solve_pressure_noalloc(nx: int, ny: int, nz: int, dx: float, params: dict, opts: Opts, dt: float,
                           eps, ux, uy, uz, p, stream=None) -> dict:
    """vos_solve_pressure_noalloc on device tensors (float64, contiguous):
    eps, ux, uy, uz are read, p is overwritten with the solution.  The library
    allocates nothing; the tensors are the caller's."""
    import torch
    for t in (eps, ux, uy, p) + ((uz,) if nz > 1 else ()):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("device float64 contiguous tensors expected")
    g = _Grid(nx, ny, nz, dx)
    pr = make_params(params)
    o = _Opts(**asdict(opts))
    st = stream if stream is not None else torch.cuda.current_stream()
    torch.cuda.current_stream().synchronize()
    dg = _Diag()
    rc = lib().vos_solve_pressure_noalloc(C.byref(g), C.byref(pr), C.byref(o), dt, C.c_void_p(eps.data_ptr()),
                                          C.c_void_p(ux.data_ptr()), C.c_void_p(uy.data_ptr()),
                                          C.c_void_p(uz.data_ptr()) if nz > 1 else None,
                                          C.c_void_p(p.data_ptr()), C.c_void_p(st.cuda_stream), C.byref(dg))
    _check(rc, diag_to_dict(dg))
    return diag_to_dict(dg)

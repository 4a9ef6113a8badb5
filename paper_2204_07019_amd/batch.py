"""Thin ctypes binding of the batch API (include/vos_batch.h): many
independent simulations advanced concurrently.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
from dataclasses import asdict
from typing import List, Optional, Sequence

import numpy as np

from . import vos

_set = False


def lib():
    global _set
    L = vos.lib()
    if not _set:
        vp = C.c_void_p
        sig = {
            "vos_batch_workspace_bytes": [C.c_int, vp, vp, C.POINTER(C.c_size_t)],
            "vos_batch_create": [C.c_int, vp, vp, vp, vp, C.c_size_t, C.c_int, C.POINTER(vp)],
            "vos_batch_destroy": [vp],
            "vos_batch_sim": [vp, C.c_int, C.POINTER(vp)],
            "vos_batch_step": [vp, vp, C.c_int, C.c_int, vp, vp],
            "vos_batch_tune": [vp, vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)],
            "vos_batch_tuning": [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_uint)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        _set = True
    return L


class Batch:
    """n simulations; ``specs`` is a list of (nx, ny, nz, dx, params dict)
    and ``opts`` one vos.Opts or a list of them."""

    def __init__(self, specs: Sequence[tuple], opts=None, workers: int = 0, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        n = len(specs)
        self.n = n
        self.specs = list(specs)
        ol = opts if isinstance(opts, (list, tuple)) else [opts or vos.Opts()] * n
        self._grids = (vos._Grid * n)(*[vos._Grid(nx, ny, nz, dx) for (nx, ny, nz, dx, _) in specs])
        self._params = (vos._Params * n)(*[vos.make_params(p) for (*_, p) in specs])
        self._opts = (vos._Opts * n)(*[vos._Opts(**asdict(o)) for o in ol])
        nbytes = C.c_size_t()
        vos._check(lib().vos_batch_workspace_bytes(n, self._grids, self._opts, C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        h = C.c_void_p()
        vos._check(lib().vos_batch_create(n, self._grids, self._params, self._opts,
                                          C.c_void_p(self.workspace.data_ptr()), nbytes.value, workers, C.byref(h)))
        self._h = h
        self.sims: List[vos.Sim] = []
        for i, (nx, ny, nz, dx, p) in enumerate(specs):
            sh = C.c_void_p()
            vos._check(lib().vos_batch_sim(self._h, i, C.byref(sh)))
            self.sims.append(vos.Sim.borrowed(sh, nx, ny, nz, dx, p, device))

    def close(self):
        if getattr(self, "_h", None):
            for s in self.sims:
                s.close()
            lib().vos_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, dt, nsteps: int = 1, freeze_solid: bool = False):
        """Advance all instances; dt is a scalar or one value per instance.
        Returns the per-instance diagnostics (dicts)."""
        n = self.n
        dts = (C.c_double * n)(*(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)).tolist()))
        dg = (vos._Diag * n)()
        st = (C.c_int * n)()
        rc = lib().vos_batch_step(self._h, dts, nsteps, vos.FREEZE_SOLID if freeze_solid else 0, dg, st)
        diags = [vos.diag_to_dict(dg[i]) for i in range(n)]
        vos._check(rc, diags)
        return diags

    def tune(self, dt, probe_steps: int = 1) -> dict:
        n = self.n
        dts = (C.c_double * n)(*(np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)).tolist()))
        w = C.c_int()
        ms = C.c_double()
        vos._check(lib().vos_batch_tune(self._h, dts, probe_steps, C.byref(w), C.byref(ms)))
        return {"workers": w.value, "best_ms": ms.value}

    def tuning(self, i: int) -> dict:
        """Instance i's tuned Krylov check interval and the level size from
        which its 2-D tiled V-cycle legs take the tall tiles."""
        ce = C.c_int()
        tb = C.c_uint()
        vos._check(lib().vos_batch_tuning(self._h, i, C.byref(ce), C.byref(tb)))
        return {"check_every": ce.value, "tile_big_cells": tb.value}

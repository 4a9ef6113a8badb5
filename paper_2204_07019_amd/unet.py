"""Thin ctypes binding of the warm-start U-Net (include/vos_unet.h).

Argument marshalling only: forward, backward and Adam run in libvos.so's
gfx950 kernels.  Tensors are torch device tensors; the network runs on a
stream of its own (default priority) unless one is given.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import vos

_set = False


class _Shape(C.Structure):
    _fields_ = [("batch", C.c_int), ("nz", C.c_int), ("ny", C.c_int), ("nx", C.c_int),
                ("cin", C.c_int), ("train", C.c_int)]


class _WarmStart(C.Structure):
    _fields_ = [("gain", C.c_double), ("use_guess", C.c_int)]


def lib():
    global _set
    L = vos.lib()
    if not _set:
        vp = C.c_void_p
        sig = {
            "vos_unet_param_count": [C.POINTER(C.c_size_t)],
            "vos_unet_workspace_bytes": [C.POINTER(_Shape), C.POINTER(C.c_size_t)],
            "vos_unet_create": [C.POINTER(_Shape), vp, C.c_size_t, vp, C.POINTER(vp)],
            "vos_unet_destroy": [vp],
            "vos_unet_set_params": [vp, vp, C.c_int],
            "vos_unet_get_params": [vp, vp, C.c_int],
            "vos_unet_get_grads": [vp, vp, C.c_int],
            "vos_unet_forward": [vp, vp, vp],
            "vos_unet_loss_grad": [vp, vp, vp, C.POINTER(C.c_double)],
            "vos_unet_adam": [vp, C.c_float, C.c_float, C.c_float, C.c_float],
            "vos_unet_train_step": [vp, vp, vp, C.c_float, C.POINTER(C.c_double)],
            "vos_attach_unet": [vp, vp, C.POINTER(_WarmStart)],
            "vos_warm_start_sample": [vp, vp, vp],
            "vos_unet_save": [vp, C.c_char_p],
            "vos_unet_load": [vp, C.c_char_p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        _set = True
    return L


def param_count() -> int:
    n = C.c_size_t()
    vos._check(lib().vos_unet_param_count(C.byref(n)))
    return int(n.value)


def workspace_bytes(batch: int, nz: int, ny: int, nx: int, cin: int = 4, train: bool = True) -> int:
    s = _Shape(batch, nz, ny, nx, cin, int(train))
    n = C.c_size_t()
    vos._check(lib().vos_unet_workspace_bytes(C.byref(s), C.byref(n)))
    return int(n.value)


class UNet:
    """Network planned for inputs (batch, nz, ny, nx, cin) FP32 NDHWC."""

    def __init__(self, batch: int, nz: int, ny: int, nx: int, cin: int = 4, train: bool = True,
                 device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.shape = (batch, nz, ny, nx)
        self.cin = cin
        self.train = train
        s = _Shape(batch, nz, ny, nx, cin, int(train))
        nbytes = C.c_size_t()
        vos._check(lib().vos_unet_workspace_bytes(C.byref(s), C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        vos._check(lib().vos_unet_create(C.byref(s), C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.n_params = param_count()

    def close(self):
        if getattr(self, "_h", None):
            lib().vos_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape, dtype=None):
        torch = self.torch
        t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a))
        t = t.to(device=self.device, dtype=dtype or torch.float32).contiguous()
        if t.numel() != int(np.prod(shape)):
            raise ValueError(f"expected {shape}, got {tuple(t.shape)}")
        torch.cuda.current_stream(self.device).synchronize()
        return t

    # ---------------------------------------------------------------- parameters
    def set_params(self, theta):
        t = self._dev(theta, (self.n_params,))
        vos._check(lib().vos_unet_set_params(self._h, C.c_void_p(t.data_ptr()), 1))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        vos._check(lib().vos_unet_get_params(self._h, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def save(self, path: str):
        """Parameters to a file (vos_unet_save)."""
        vos._check(lib().vos_unet_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """Parameters from a file written by save (vos_unet_load)."""
        vos._check(lib().vos_unet_load(self._h, os.fsencode(path)))

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        vos._check(lib().vos_unet_get_grads(self._h, out.ctypes.data_as(C.c_void_p), 0))
        return out

    # ---------------------------------------------------------------- compute
    def forward(self, x):
        """x: (batch, nz, ny, nx, cin) -> y (batch, nz, ny, nx) float32 device tensor."""
        xt = self._dev(x, self.shape + (self.cin,))
        y = self.torch.empty(self.shape, dtype=self.torch.float32, device=self.device)
        self.torch.cuda.current_stream(self.device).synchronize()
        vos._check(lib().vos_unet_forward(self._h, C.c_void_p(xt.data_ptr()), C.c_void_p(y.data_ptr())))
        self.stream.synchronize()
        return y

    def loss_grad(self, x, target) -> float:
        xt = self._dev(x, self.shape + (self.cin,))
        tt = self._dev(target, self.shape)
        loss = C.c_double()
        vos._check(lib().vos_unet_loss_grad(self._h, C.c_void_p(xt.data_ptr()), C.c_void_p(tt.data_ptr()),
                                            C.byref(loss)))
        return loss.value

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        vos._check(lib().vos_unet_adam(self._h, lr, beta1, beta2, eps))
        self.stream.synchronize()

    def train_step(self, x, target, lr: float, want_loss: bool = True) -> Optional[float]:
        """One Adam step on (x, target); x and target should already be
        contiguous float32 device tensors for speed."""
        xt = self._dev(x, self.shape + (self.cin,)) if not _ready(x, self) else x
        tt = self._dev(target, self.shape) if not _ready(target, self) else target
        loss = C.c_double()
        vos._check(lib().vos_unet_train_step(self._h, C.c_void_p(xt.data_ptr()), C.c_void_p(tt.data_ptr()), lr,
                                             C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


def _ready(t, net) -> bool:
    torch = net.torch
    return isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()


def attach(sim: "vos.Sim", net: Optional[UNet], gain: float = 1.0, use_guess: bool = True):
    """Attach a network (batch 1, the simulation's grid, cin 4) as the
    pressure solve's warm start, or detach it (net=None)."""
    ws = _WarmStart(gain, int(use_guess))
    vos._check(lib().vos_attach_unet(sim._h, net._h if net is not None else None, C.byref(ws)))
    sim._unet = net


def warm_start_sample(sim: "vos.Sim"):
    """(input (nz, ny, nx, 4), target (nz, ny, nx)) of the last step's pressure solve."""
    torch = sim.torch
    nz, ny, nx = sim.shape
    x = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=sim.device)
    t = torch.empty((nz, ny, nx), dtype=torch.float32, device=sim.device)
    torch.cuda.current_stream(sim.device).synchronize()
    vos._check(lib().vos_warm_start_sample(sim._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr())))
    return x, t

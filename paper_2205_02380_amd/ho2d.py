"""Python binding of ``include/chasm_ho2d.h`` (ctypes): the 2-D harmonic-oscillator
workload of Sec. 5.1 (LPC1 with spline x-advection and spectral k-derivative, FP64).
Argument marshalling only."""
from __future__ import annotations

import ctypes
from typing import Optional

from . import chasm

EXPORTS = ("chasm_ho2d_create", "chasm_ho2d_step", "chasm_ho2d_destroy")
_bound = False


class chasm_ho2d_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("x_lo", ctypes.c_double), ("hx", ctypes.c_double),
                ("nk", ctypes.c_int32), ("k_lo", ctypes.c_double), ("hk", ctypes.c_double),
                ("patch", ctypes.c_int32), ("ghost", ctypes.c_int32),
                ("omega", ctypes.c_double), ("tau", ctypes.c_double), ("inflow", ctypes.c_int32)]


def lib():
    global _bound
    L = chasm.lib()
    if not _bound:
        vp = ctypes.c_void_p
        L.chasm_ho2d_create.argtypes = [ctypes.POINTER(chasm_ho2d_desc), vp, vp, ctypes.POINTER(vp)]
        L.chasm_ho2d_step.argtypes = [vp, ctypes.c_int32]
        L.chasm_ho2d_destroy.argtypes = [vp]
        for n in EXPORTS:
            getattr(L, n).restype = ctypes.c_int
        _bound = True
    return L


def _check(st: int) -> None:
    if st != chasm.CHASM_OK:
        raise chasm.ChasmError(st, chasm.chasm_advect_last_error())


INFLOW = {"zero": 0, "extrapolate": 1}


def make_desc(nx, x_lo, hx, nk, k_lo, hk, patch, ghost, omega, tau, inflow: str = "zero") -> chasm_ho2d_desc:
    return chasm_ho2d_desc(int(nx), float(x_lo), float(hx), int(nk), float(k_lo), float(hk), int(patch), int(ghost),
                           float(omega), float(tau), INFLOW[inflow])


def chasm_ho2d_create(desc: chasm_ho2d_desc, f_dev: int, hip_stream: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().chasm_ho2d_create(ctypes.byref(desc), ctypes.c_void_p(f_dev), ctypes.c_void_p(hip_stream),
                                   ctypes.byref(h)))
    return h.value


def chasm_ho2d_step(h: int, nsteps: int) -> None:
    _check(lib().chasm_ho2d_step(ctypes.c_void_p(h), int(nsteps)))


def chasm_ho2d_destroy(h: Optional[int]) -> None:
    _check(lib().chasm_ho2d_destroy(ctypes.c_void_p(h)))


class HO2D:
    """Advance f[k][x] (contiguous float64 device tensor) in place."""

    def __init__(self, f, nx, x_lo, hx, nk, k_lo, hk, patch, ghost, omega, tau, inflow: str = "zero", stream=None):
        import torch
        if not f.is_cuda or not f.is_contiguous() or f.dtype != torch.float64 or f.numel() != nx * nk:
            raise ValueError("f must be a contiguous float64 device tensor of nk x nx")
        self.f = f
        self.stream = stream if stream is not None else torch.cuda.current_stream(f.device)
        self.h = chasm_ho2d_create(make_desc(nx, x_lo, hx, nk, k_lo, hk, patch, ghost, omega, tau, inflow),
                                   f.data_ptr(), self.stream.cuda_stream)

    def step(self, n: int = 1) -> None:
        chasm_ho2d_step(self.h, n)

    def close(self) -> None:
        if self.h:
            chasm_ho2d_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

"""Python binding of the C ABI in ``include/chasm_lpc1.h`` (ctypes): the LPC1 time step
(Sec. 2.2) of the Wigner-Coulomb equation, advection plus truncated-kernel Theta_V.
Argument marshalling only; every step runs in ``libchasm.so``."""
from __future__ import annotations

import ctypes
from typing import Optional

from . import chasm, theta
from .inputs import Grid

EXPORTS = ("chasm_lpc1_create", "chasm_lpc1_step", "chasm_lpc1_destroy")
_bound = False


def lib():
    global _bound
    L = theta.lib()
    if not _bound:
        vp = ctypes.c_void_p
        L.chasm_lpc1_create.argtypes = [ctypes.POINTER(chasm.chasm_advect_desc), ctypes.POINTER(theta.chasm_theta_desc),
                                        vp, vp, ctypes.POINTER(vp)]
        L.chasm_lpc1_step.argtypes = [vp, ctypes.c_int32]
        L.chasm_lpc1_destroy.argtypes = [vp]
        for n in EXPORTS:
            getattr(L, n).restype = ctypes.c_int
        _bound = True
    return L


def _check(st: int) -> None:
    if st != chasm.CHASM_OK:
        raise chasm.ChasmError(st, chasm.chasm_advect_last_error())


def chasm_lpc1_create(adv: chasm.chasm_advect_desc, th: theta.chasm_theta_desc, f_dev: int, hip_stream: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().chasm_lpc1_create(ctypes.byref(adv), ctypes.byref(th), ctypes.c_void_p(f_dev),
                                   ctypes.c_void_p(hip_stream), ctypes.byref(h)))
    return h.value


def chasm_lpc1_step(h: int, nsteps: int) -> None:
    _check(lib().chasm_lpc1_step(ctypes.c_void_p(h), int(nsteps)))


def chasm_lpc1_destroy(h: Optional[int]) -> None:
    _check(lib().chasm_lpc1_destroy(ctypes.c_void_p(h)))


class LPC1:
    """Advance ``f`` (contiguous device tensor of ``grid``, float32/float64) in place by
    LPC1 steps of size tau with V = -sum_a z_a / |x - x_a|."""

    def __init__(self, f, grid: Grid, patch, ghost: int, tau: float, nuclei, charges=None, closure: str = "pmbc",
                 schedule: str = "auto", stream=None):
        import torch
        if not f.is_cuda or not f.is_contiguous() or f.numel() != grid.points:
            raise ValueError("f must be one contiguous device field of the grid")
        dtype = {torch.float32: "f32", torch.float64: "f64"}[f.dtype]
        self.f = f
        self.stream = stream if stream is not None else torch.cuda.current_stream(f.device)
        adv = chasm.make_desc(grid, patch, ghost, tau, dtype, closure, 1, 0, schedule)
        th = theta.make_desc(grid, nuclei, charges, dtype, 1)
        self.h = chasm_lpc1_create(adv, th, f.data_ptr(), self.stream.cuda_stream)

    def step(self, n: int = 1) -> None:
        chasm_lpc1_step(self.h, n)

    def close(self) -> None:
        if self.h:
            chasm_lpc1_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

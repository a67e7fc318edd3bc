"""Python binding of the C ABI in ``include/chasm_theta.h`` (ctypes): the truncated-kernel
evaluation of the Coulomb pseudo-differential operator Theta_V (Sec. 4).

Argument marshalling only: the convolutions run in ``libchasm.so``'s HIP kernels and
the tensor of eq. 4.9 is built by the library's host code.  No fallback.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import chasm
from .inputs import Grid

MAX_NUCLEI = 4


class chasm_theta_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32 * 3),
        ("nk", ctypes.c_int32 * 3),
        ("x_lo", ctypes.c_double * 3),
        ("x_hi", ctypes.c_double * 3),
        ("k_lo", ctypes.c_double * 3),
        ("k_hi", ctypes.c_double * 3),
        ("nnuc", ctypes.c_int32),
        ("x_nuc", (ctypes.c_double * 3) * MAX_NUCLEI),
        ("z_nuc", ctypes.c_double * MAX_NUCLEI),
        ("dtype", ctypes.c_int32),
        ("nbatch", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


FLAG_STAGED = 1


EXPORTS = ("chasm_theta_create", "chasm_theta_apply", "chasm_theta_workspace_bytes", "chasm_theta_tensor",
           "chasm_theta_destroy")

_bound = False


def lib():
    global _bound
    L = chasm.lib()
    if not _bound:
        vp = ctypes.c_void_p
        pd = ctypes.POINTER(chasm_theta_desc)
        L.chasm_theta_create.argtypes = [pd, vp, ctypes.POINTER(vp)]
        L.chasm_theta_apply.argtypes = [vp, vp, vp]
        L.chasm_theta_workspace_bytes.argtypes = [pd, ctypes.POINTER(ctypes.c_size_t)]
        L.chasm_theta_tensor.argtypes = [pd, ctypes.POINTER(ctypes.c_double)]
        L.chasm_theta_destroy.argtypes = [vp]
        for n in EXPORTS:
            getattr(L, n).restype = ctypes.c_int
        _bound = True
    return L


def _check(st: int) -> None:
    if st != chasm.CHASM_OK:
        raise chasm.ChasmError(st, chasm.chasm_advect_last_error())


def make_desc(grid: Grid, nuclei: Sequence[Sequence[float]], charges: Optional[Sequence[float]] = None,
              dtype: str = "f32", nbatch: int = 1, staged: bool = False) -> chasm_theta_desc:
    d = chasm_theta_desc()
    for a in range(3):
        d.nx[a], d.nk[a] = int(grid.nx[a]), int(grid.nk[a])
        d.x_lo[a], d.x_hi[a] = float(grid.x_lo[a]), float(grid.x_hi[a])
        d.k_lo[a], d.k_hi[a] = float(grid.k_lo[a]), float(grid.k_hi[a])
    charges = [1.0] * len(nuclei) if charges is None else list(charges)
    d.nnuc = len(nuclei)
    for i, (x, z) in enumerate(zip(nuclei, charges)):
        if i >= MAX_NUCLEI:
            break
        for a in range(3):
            d.x_nuc[i][a] = float(x[a])
        d.z_nuc[i] = float(z)
    d.dtype = {"f32": chasm.CHASM_F32, "f64": chasm.CHASM_F64}[dtype]
    d.nbatch = int(nbatch)
    d.flags = FLAG_STAGED if staged else 0
    return d


def chasm_theta_create(desc: chasm_theta_desc, hip_stream: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().chasm_theta_create(ctypes.byref(desc), ctypes.c_void_p(hip_stream), ctypes.byref(h)))
    return h.value


def chasm_theta_apply(h: int, f_dev: int, out_dev: int) -> None:
    _check(lib().chasm_theta_apply(ctypes.c_void_p(h), ctypes.c_void_p(f_dev), ctypes.c_void_p(out_dev)))


def chasm_theta_workspace_bytes(desc: chasm_theta_desc) -> int:
    b = ctypes.c_size_t()
    _check(lib().chasm_theta_workspace_bytes(ctypes.byref(desc), ctypes.byref(b)))
    return b.value


def chasm_theta_tensor(desc: chasm_theta_desc) -> np.ndarray:
    """T_p of eq. 4.9 as the library builds it, [p3][p2][p1] over |p_d| <= nk_d - 1."""
    shape = tuple(2 * int(desc.nk[a]) - 1 for a in (2, 1, 0))
    out = np.zeros(shape)
    _check(lib().chasm_theta_tensor(ctypes.byref(desc), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def chasm_theta_destroy(h: Optional[int]) -> None:
    _check(lib().chasm_theta_destroy(ctypes.c_void_p(h)))


class Theta:
    """out = Theta_V^T[f] for V = -sum_a z_a / |x - x_a|, on fields of ``grid``
    (torch device tensors [b][k3][k2][k1][x3][x2][x1] or without b)."""

    def __init__(self, grid: Grid, nuclei, charges=None, dtype: str = "f32", nbatch: int = 1, stream=None,
                 staged: bool = False):
        import torch
        self.grid = grid
        self.desc = make_desc(grid, nuclei, charges, dtype, nbatch, staged)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = chasm_theta_create(self.desc, self.stream.cuda_stream)
        self.nbatch = nbatch
        self.dtype = dtype

    def apply(self, f, out=None):
        import torch
        want = {"f32": torch.float32, "f64": torch.float64}[self.dtype]
        n = self.grid.points * self.nbatch
        if out is None:
            out = torch.empty_like(f)
        for t in (f, out):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != want or t.numel() != n:
                raise ValueError("f and out must be contiguous device tensors of the handle's grid and dtype")
        chasm_theta_apply(self.h, f.data_ptr(), out.data_ptr())
        return out

    def close(self) -> None:
        if self.h:
            chasm_theta_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Python binding of the C ABI in ``include/chasm_advect.h`` (ctypes).

Argument marshalling only: every step of the advection runs in ``libchasm.so``'s HIP
kernels.  PyTorch supplies device memory (the caller's field tensor) and the stream.
If the library is not built the first call raises; there is no fallback.

The functions named ``chasm_advect_*`` mirror the C entry points one to one;
``Advect`` is a small owning wrapper around a handle.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from .inputs import Grid

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchasm.so")

CHASM_OK, CHASM_EINVAL, CHASM_ENOMEM, CHASM_EDEVICE, CHASM_ESTATE, CHASM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CHASM_F32, CHASM_F64 = 0, 1
CHASM_CLOSURE_PMBC, CHASM_CLOSURE_POLY3, CHASM_CLOSURE_NEUMANN, CHASM_CLOSURE_HERMITE = 0, 1, 2, 3
CHASM_SCHED_AUTO, CHASM_SCHED_CUBE, CHASM_SCHED_SLAB, CHASM_SCHED_PLAIN = 0, 1, 2, 3
CHASM_FLAG_REDUCE_EACH_STEP, CHASM_FLAG_GRAPH, CHASM_FLAG_OUT_OF_PLACE, CHASM_FLAG_RUNTIME_SHAPE = 1, 2, 4, 8
CHASM_FLAG_TILE_SHIFT, CHASM_FLAG_TILE_MASK = 4, 3 << 4
CHASM_FLAG_OBSERVE = 1 << 6
TILES = (0, 1, 2)


def CHASM_FLAG_TILE(t: int) -> int:
    """Launch-shape variant t of the compiled SLAB and PLAIN passes (0 default)."""
    return int(t) << CHASM_FLAG_TILE_SHIFT

SCHEDULES = {"auto": 0, "cube": 1, "slab": 2, "plain": 3}
SCHEDULE_NAMES = {v: k for k, v in SCHEDULES.items()}
CLOSURES = {"pmbc": 0, "poly3": 1, "neumann": 2, "hermite": 3}
NRED = 8
DIAG_NAMES = ("mass", "l2", "x1", "x2", "x3", "k1", "k2", "k3")


class ChasmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"chasm status {status}: {msg}")
        self.status = status


class chasm_advect_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32 * 3),
        ("nk", ctypes.c_int32 * 3),
        ("x_lo", ctypes.c_double * 3),
        ("x_hi", ctypes.c_double * 3),
        ("k_lo", ctypes.c_double * 3),
        ("k_hi", ctypes.c_double * 3),
        ("patch", ctypes.c_int32 * 3),
        ("ghost", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("dtype", ctypes.c_int32),
        ("closure", ctypes.c_int32),
        ("nbatch", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("schedule", ctypes.c_int32),
        ("history_cap", ctypes.c_int32),
        ("slope_lo", ctypes.c_double * 3),
        ("slope_hi", ctypes.c_double * 3),
    ]


EXPORTS = (
    "chasm_advect_create", "chasm_advect_step", "chasm_advect_mass", "chasm_advect_diagnostics",
    "chasm_advect_history", "chasm_advect_step_many", "chasm_advect_workspace_bytes", "chasm_advect_schedule",
    "chasm_advect_destroy", "chasm_advect_last_error", "chasm_advect_version", "chasm_advect_marginals",
    "chasm_advect_diagnostics_noalloc", "chasm_advect_observables",
)

_lib = None


def lib():
    """Load libchasm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2205_02380_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, pd = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)
    pdesc = ctypes.POINTER(chasm_advect_desc)
    L.chasm_advect_create.argtypes = [pdesc, vp, vp, ctypes.POINTER(vp)]
    L.chasm_advect_step.argtypes = [vp, i32]
    L.chasm_advect_mass.argtypes = [vp, pd, pd, pd]
    L.chasm_advect_diagnostics.argtypes = [vp, pd]
    L.chasm_advect_history.argtypes = [vp, pd, i32, ctypes.POINTER(i32)]
    L.chasm_advect_step_many.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32)]
    L.chasm_advect_workspace_bytes.argtypes = [pdesc, ctypes.POINTER(ctypes.c_size_t)]
    L.chasm_advect_schedule.argtypes = [vp, ctypes.POINTER(i32)]
    L.chasm_advect_destroy.argtypes = [vp]
    L.chasm_advect_marginals.argtypes = [vp, pd, pd, pd, pd]
    L.chasm_advect_observables.argtypes = [vp, pd, pd, pd, pd]
    L.chasm_advect_diagnostics_noalloc.argtypes = [pdesc, vp, vp, vp]
    L.chasm_advect_last_error.restype = ctypes.c_char_p
    L.chasm_advect_version.restype = ctypes.c_char_p
    for name in ("create", "step", "mass", "diagnostics", "history", "step_many", "workspace_bytes", "schedule",
                 "destroy", "marginals", "diagnostics_noalloc", "observables"):
        getattr(L, "chasm_advect_" + name).restype = ctypes.c_int
    _lib = L
    return L


def _check(st: int) -> None:
    if st != CHASM_OK:
        raise ChasmError(st, lib().chasm_advect_last_error().decode())


def make_desc(grid: Grid, patch, ghost: int, dt: float, dtype: str = "f32", closure: str = "pmbc",
              nbatch: int = 1, flags: int = 0, schedule: str = "auto", history_cap: int = 0,
              slopes=None) -> chasm_advect_desc:
    """slopes: ((lo1, hi1), (lo2, hi2), (lo3, hi3)) end slopes of the Hermite closure."""
    if isinstance(patch, int):
        patch = (patch, patch, patch)
    d = chasm_advect_desc()
    for a in range(3):
        d.nx[a] = int(grid.nx[a])
        d.nk[a] = int(grid.nk[a])
        d.x_lo[a], d.x_hi[a] = float(grid.x_lo[a]), float(grid.x_hi[a])
        d.k_lo[a], d.k_hi[a] = float(grid.k_lo[a]), float(grid.k_hi[a])
        d.patch[a] = int(patch[a])
    d.ghost = int(ghost)
    d.dt = float(dt)
    d.dtype = {"f32": CHASM_F32, "f64": CHASM_F64}[dtype]
    d.closure = CLOSURES[closure]
    d.nbatch = int(nbatch)
    d.flags = int(flags)
    d.schedule = SCHEDULES[schedule]
    d.history_cap = int(history_cap)
    if slopes is not None:
        for a in range(3):
            d.slope_lo[a], d.slope_hi[a] = float(slopes[a][0]), float(slopes[a][1])
    return d


# ---- the C entry points, one to one ---------------------------------------------
def chasm_advect_create(desc: chasm_advect_desc, f_dev: int, hip_stream: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().chasm_advect_create(ctypes.byref(desc), ctypes.c_void_p(f_dev), ctypes.c_void_p(hip_stream),
                                     ctypes.byref(h)))
    return h.value


def chasm_advect_step(h: int, nsteps: int) -> None:
    _check(lib().chasm_advect_step(ctypes.c_void_p(h), int(nsteps)))


def chasm_advect_mass(h: int):
    m, l2 = ctypes.c_double(), ctypes.c_double()
    mom = (ctypes.c_double * 6)()
    _check(lib().chasm_advect_mass(ctypes.c_void_p(h), ctypes.byref(m), ctypes.byref(l2), mom))
    return m.value, l2.value, np.array(mom[:])


def chasm_advect_diagnostics(h: int, nbatch: int) -> np.ndarray:
    out = np.zeros((nbatch, NRED))
    _check(lib().chasm_advect_diagnostics(ctypes.c_void_p(h), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def chasm_advect_diagnostics_noalloc(desc: chasm_advect_desc, f_dev: int, hip_stream: int, out_dev: int) -> None:
    """Allocation-free diagnostics of the field at f_dev into the device buffer out_dev
    (nbatch*8 doubles); asynchronous on hip_stream."""
    _check(lib().chasm_advect_diagnostics_noalloc(ctypes.byref(desc), ctypes.c_void_p(f_dev),
                                                  ctypes.c_void_p(hip_stream), ctypes.c_void_p(out_dev)))


def chasm_advect_history(h: int, nbatch: int, max_steps: int) -> np.ndarray:
    out = np.zeros((max(max_steps, 1), nbatch, NRED))
    n = ctypes.c_int32()
    _check(lib().chasm_advect_history(ctypes.c_void_p(h), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      int(max_steps), ctypes.byref(n)))
    return out[: n.value]


def chasm_advect_step_many(hs: Sequence[int], nsteps: Sequence[int]) -> None:
    n = len(hs)
    arr = (ctypes.c_void_p * max(n, 1))(*hs)
    st = (ctypes.c_int32 * max(n, 1))(*[int(s) for s in nsteps])
    _check(lib().chasm_advect_step_many(arr, n, st))


def chasm_advect_marginals(h: int, grid: Grid, nbatch: int):
    """(W1, W2, W3, P): arrays [b][k_d][x_d] for W_d and [b][x2][x1] for P (FP64)."""
    ws = [np.zeros((nbatch, grid.nk[d], grid.nx[d])) for d in range(3)]
    p = np.zeros((nbatch, grid.nx[1], grid.nx[0]))
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().chasm_advect_marginals(ctypes.c_void_p(h), ptr(ws[0]), ptr(ws[1]), ptr(ws[2]), ptr(p)))
    return ws[0], ws[1], ws[2], p


def chasm_advect_observables(h: int, grid: Grid, nbatch: int):
    """(W1, W2, W3, P) formed in the last observed step call (CHASM_FLAG_OBSERVE)."""
    ws = [np.zeros((nbatch, grid.nk[d], grid.nx[d])) for d in range(3)]
    p = np.zeros((nbatch, grid.nx[1], grid.nx[0]))
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(lib().chasm_advect_observables(ctypes.c_void_p(h), ptr(ws[0]), ptr(ws[1]), ptr(ws[2]), ptr(p)))
    return ws[0], ws[1], ws[2], p


def chasm_advect_workspace_bytes(desc: chasm_advect_desc) -> int:
    b = ctypes.c_size_t()
    _check(lib().chasm_advect_workspace_bytes(ctypes.byref(desc), ctypes.byref(b)))
    return b.value


def chasm_advect_schedule(h: int) -> str:
    s = ctypes.c_int32()
    _check(lib().chasm_advect_schedule(ctypes.c_void_p(h), ctypes.byref(s)))
    return SCHEDULE_NAMES[s.value]


def chasm_advect_destroy(h: Optional[int]) -> None:
    _check(lib().chasm_advect_destroy(ctypes.c_void_p(h)))


def chasm_advect_last_error() -> str:
    return lib().chasm_advect_last_error().decode()


def chasm_advect_version() -> str:
    return lib().chasm_advect_version().decode()


# ---- owning wrapper ------------------------------------------------------------
class Advect:
    """A handle advancing ``f`` (a contiguous CUDA/HIP torch tensor of shape
    [b][k3][k2][k1][x3][x2][x1] or without b); every step ends in ``f``.  With
    ``out_of_place`` the sweeps go through a second, library-owned field; ``tile``
    selects the launch-shape variant of the SLAB and PLAIN passes (FP32 48^3 / 64^3)."""

    def __init__(self, f, grid: Grid, patch, ghost: int, dt: float, closure: str = "pmbc",
                 schedule: str = "auto", reduce_each_step: bool = False, graph: bool = False,
                 history_cap: int = 0, stream=None, out_of_place: bool = False, runtime_shape: bool = False,
                 slopes=None, tile: int = 0, observe: bool = False):
        import torch
        if not f.is_cuda or not f.is_contiguous():
            raise ValueError("f must be a contiguous device tensor")
        dtype = {torch.float32: "f32", torch.float64: "f64"}.get(f.dtype)
        if dtype is None:
            raise ValueError("f must be float32 or float64")
        cube = grid.cube * grid.nkpts
        if f.numel() % cube:
            raise ValueError("f does not hold whole fields of this grid")
        nbatch = f.numel() // cube
        flags = ((CHASM_FLAG_REDUCE_EACH_STEP if reduce_each_step else 0) | (CHASM_FLAG_GRAPH if graph else 0)
                 | (CHASM_FLAG_OUT_OF_PLACE if out_of_place else 0)
                 | (CHASM_FLAG_RUNTIME_SHAPE if runtime_shape else 0) | CHASM_FLAG_TILE(tile)
                 | (CHASM_FLAG_OBSERVE if observe else 0))
        self.desc = make_desc(grid, patch, ghost, dt, dtype, closure, nbatch, flags, schedule, history_cap, slopes)
        self.f = f
        self.nbatch = nbatch
        self.grid = grid
        self.stream = stream if stream is not None else torch.cuda.current_stream(f.device)
        self.h = chasm_advect_create(self.desc, f.data_ptr(), self.stream.cuda_stream)

    def step(self, n: int = 1) -> None:
        chasm_advect_step(self.h, n)

    def mass(self):
        return chasm_advect_mass(self.h)

    def diagnostics(self) -> np.ndarray:
        return chasm_advect_diagnostics(self.h, self.nbatch)

    def marginals(self):
        """Reduced Wigner functions W1, W2, W3 ([b][k_d][x_d]) and the spatial marginal
        P ([b][x2][x1]) of the current field (Sec. 5), FP64."""
        return chasm_advect_marginals(self.h, self.grid, self.nbatch)

    def observables(self):
        """(W1, W2, W3, P) formed by the last sweep of the last step call (``observe``)."""
        return chasm_advect_observables(self.h, self.grid, self.nbatch)

    def history(self, max_steps: int = 1 << 20) -> np.ndarray:
        return chasm_advect_history(self.h, self.nbatch, max_steps)

    @property
    def schedule(self) -> str:
        return chasm_advect_schedule(self.h)

    def close(self) -> None:
        if self.h:
            chasm_advect_destroy(self.h)
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


def step_many(advects: Sequence[Advect], nsteps: Sequence[int]) -> None:
    chasm_advect_step_many([a.h for a in advects], nsteps)


def supported(grid: Grid, patch, ghost: int, dt: float = 0.0, dtype: str = "f32", closure: str = "pmbc",
              schedule: str = "auto", tile: int = 0) -> bool:
    """True when the library accepts this grid / patch / ghost / dtype / closure and
    schedule (asks the library's own descriptor validation; no device work).  Every
    valid descriptor is accepted with schedule 'auto' or 'plain' unless a resource
    limit is hit; 'cube' and 'slab' need compiled kernels."""
    try:
        chasm_advect_workspace_bytes(make_desc(grid, patch, ghost, dt, dtype, closure,
                                               flags=CHASM_FLAG_TILE(tile), schedule=schedule))
        return True
    except ChasmError:
        return False


def compiled_shapes(sizes=(8, 16, 24, 32, 48, 64)) -> list:
    """Every (dtype, N, M, ghost, closure) with compiled kernels, for cubic x-grids of N
    nodes per axis (found through descriptor validation: only compiled shapes offer the
    SLAB schedule)."""
    out = []
    for n in sizes:
        grid = Grid((n, n, n), (0.0,) * 3, (float(n),) * 3, (1, 1, 1), (0.0,) * 3, (1.0,) * 3)
        for dt in ("f32", "f64"):
            for cl in ("pmbc", "poly3", "neumann"):
                for m in range(2, n + 1):
                    for g in range(1, n):
                        if supported(grid, m, g, 0.0, dt, cl, "slab"):
                            out.append((dt, n, m, g, cl))
    return out

"""FP64 CPU oracle for the CHASM characteristic (spatial-advection) step.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` import this package.  It shares no code with
the HIP library (``paper_2205_02380_amd``); the only module both sides use is the
seeded input generator, which holds none of the method's arithmetic.

The arithmetic lives in ``chasm_oracle.c`` (plain C, FP64, OpenMP over k-points);
this module is a ctypes binding over numpy arrays.  Paper: Xiong, Zhang, Shao,
arXiv:2205.02380; section/equation citations are on each function.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chasm_oracle.c")
_LIB = os.path.join(_HERE, "libchasm_oracle.so")

PMBC = 0    # paper closure: truncated rows of the natural-BC inverse (eqs. 3.4-3.5)
POLY3 = 1   # cubic-exact variant of those rows (not in the paper; see module docstring of the C file)
NEUMANN = 2  # rows of the inverse of the zero-slope Hermite (Neumann) global matrix (eq. 2.13)
HERMITE = 3  # the Hermite global matrix (eq. 2.13) with given end slopes phi_L, phi_R

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, IEEE FP64, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # CHASM_ORACLE_LIB: a build of the same source made elsewhere (the sanitizer run)
    path = os.environ.get("CHASM_ORACLE_LIB")
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
    lib = ctypes.CDLL(path)
    d, i, pd, pi = ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.chasm_oracle_bspline.restype = d
    lib.chasm_oracle_bspline.argtypes = [d]
    lib.chasm_oracle_npatch.argtypes = [i, i]
    lib.chasm_oracle_natural_inverse.argtypes = [i, d, pd]
    lib.chasm_oracle_stencils.argtypes = [i, i, i, d, i, pd]
    lib.chasm_oracle_interface_derivs.argtypes = [i, i, pd, pd, pd]
    lib.chasm_oracle_line_coefficients.argtypes = [i, i, d, i, pd, pd, pd]
    lib.chasm_oracle_line.argtypes = [i, i, d, i, pd, d, pd, pd]
    lib.chasm_oracle_global_line.argtypes = [i, d, d, pd, pd]
    lib.chasm_oracle_global_line_bc.argtypes = [i, d, i, d, pd, pd]
    lib.chasm_oracle_global_inverse.argtypes = [i, d, i, pd]
    lib.chasm_oracle_advect6d.argtypes = [pi, pd, pi, pd, pd, pi, i, i, d, i, i, pi, pd, i]
    lib.chasm_oracle_advect6d_bc.argtypes = [pi, pd, pi, pd, pd, pi, i, i, pd, pd, d, i, i, pi, pd, i]
    lib.chasm_oracle_stencils_bc.argtypes = [i, i, i, d, i, d, d, pd, pd]
    lib.chasm_oracle_line_bc.argtypes = [i, i, d, i, pd, pd, d, pd, pd]
    lib.chasm_oracle_global_line_hermite.argtypes = [i, d, d, d, d, pd, pd]
    lib.chasm_oracle_reduce.argtypes = [pi, pd, pd, pi, pd, pd, i, pd, pd]
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} failed (rc={rc})")


def bspline(t: float) -> float:
    """Cubic B-spline centred at 0 (eq. 2.10 with x = x_nu + t h)."""
    return _load().chasm_oracle_bspline(float(t))


def npatch(N: int, M: int) -> int:
    """Patches of M cells covering N nodes: p = ceil((N-1)/M) (Sec. 3.1, eq. 3.1)."""
    return _load().chasm_oracle_npatch(N, M)


def natural_inverse(N: int, h: float) -> np.ndarray:
    """Inverse of the natural-BC global spline matrix (Sec. 3.1.2, eq. 3.5's A-tilde).
    Row/column u corresponds to eta_{u-1}; data phi_j is column j+1."""
    out = np.zeros((N + 2, N + 2))
    _check(_load().chasm_oracle_natural_inverse(N, float(h), _dp(out)), "natural_inverse")
    return out


def stencils(N: int, M: int, g: int, h: float, closure: int = PMBC) -> np.ndarray:
    """Interface stencil rows c_j(I) (eqs. 3.4-3.5), (p+1) x N dense with zeros off-band."""
    p = npatch(N, M)
    out = np.zeros((p + 1, N))
    _check(_load().chasm_oracle_stencils(N, M, g, float(h), closure, _dp(out)), "stencils")
    return out


def stencils_bc(N: int, M: int, g: int, h: float, closure: int = PMBC, slopes=(0.0, 0.0)):
    """Interface rows and, for closure HERMITE, the end-slope part of each interface
    slope (eq. 2.13 columns of the global inverse, truncated): (c, bias)."""
    p = npatch(N, M)
    c = np.zeros((p + 1, N))
    bias = np.zeros(p + 1)
    _check(_load().chasm_oracle_stencils_bc(N, M, g, float(h), closure, float(slopes[0]), float(slopes[1]), _dp(c),
                                            _dp(bias)), "stencils_bc")
    return c, bias


def line_bc(N: int, M: int, g: int, h: float, alpha: float, phi, closure: int = HERMITE,
            slopes=(0.0, 0.0)) -> np.ndarray:
    """One patched sweep of one line with the end slopes of closure HERMITE."""
    c, bias = stencils_bc(N, M, g, h, closure, slopes)
    phi = _f64(phi)
    out = np.zeros(N)
    _check(_load().chasm_oracle_line_bc(N, M, float(h), closure, _dp(c), _dp(bias), float(alpha), _dp(phi),
                                        _dp(out)), "line_bc")
    return out


def global_line_hermite(N: int, h: float, alpha: float, phi, slopes=(0.0, 0.0)) -> np.ndarray:
    """Brute-force global spline with the Hermite rows of eq. 2.13 and given end slopes."""
    phi = _f64(phi)
    out = np.zeros(N)
    _check(_load().chasm_oracle_global_line_hermite(N, float(h), float(slopes[0]), float(slopes[1]), float(alpha),
                                                    _dp(phi), _dp(out)), "global_line_hermite")
    return out


def interface_derivs(N: int, M: int, c: np.ndarray, phi) -> np.ndarray:
    p = npatch(N, M)
    c = _f64(c)
    phi = _f64(phi)
    out = np.zeros(p + 1)
    _check(_load().chasm_oracle_interface_derivs(N, M, _dp(c), _dp(phi), _dp(out)), "interface_derivs")
    return out


def line_coefficients(N: int, M: int, h: float, c: np.ndarray, phi, closure: int = PMBC) -> np.ndarray:
    """Per-patch coefficients eta^{(l)}_{nu}, nu = -2..M+2 at column nu+2 (Sec. 3.1.2 step 5)."""
    p = npatch(N, M)
    c = _f64(c)
    phi = _f64(phi)
    out = np.zeros((p, M + 5))
    _check(_load().chasm_oracle_line_coefficients(N, M, float(h), closure, _dp(c), _dp(phi), _dp(out)),
           "line_coefficients")
    return out


def line(N: int, M: int, g: int, h: float, alpha: float, phi, closure: int = PMBC,
         c: np.ndarray | None = None) -> np.ndarray:
    """One patched sweep of one line: f_new(x_j) = s(x_j - alpha h) (Sec. 3.1)."""
    if c is None:
        c = stencils(N, M, g, h, closure)
    c = _f64(c)
    phi = _f64(phi)
    out = np.zeros(N)
    _check(_load().chasm_oracle_line(N, M, float(h), closure, _dp(c), float(alpha), _dp(phi), _dp(out)), "line")
    return out


def global_line(N: int, h: float, alpha: float, phi, bc: int = 0) -> np.ndarray:
    """Brute-force reference: the global spline of the whole line, no patches, with the
    natural boundary rows (bc 0, eq. 2.14) or the zero-slope Hermite rows (bc 1, the
    Neumann condition of eq. 2.13 with phi_L = phi_R = 0)."""
    phi = _f64(phi)
    out = np.zeros(N)
    _check(_load().chasm_oracle_global_line_bc(N, float(h), int(bc), float(alpha), _dp(phi), _dp(out)),
           "global_line")
    return out


def global_inverse(N: int, h: float, bc: int) -> np.ndarray:
    """Inverse of the global spline matrix with natural (bc 0) or Neumann (bc 1) rows."""
    out = np.zeros((N + 2, N + 2))
    _check(_load().chasm_oracle_global_inverse(N, float(h), int(bc), _dp(out)), "global_inverse")
    return out


def advect6d(cubes: np.ndarray, nx, hx, nk, klo, hk, M, g: int, dt: float, nsteps: int,
             closure: int = PMBC, kidx=None, nthreads: int = 0, slopes=None) -> np.ndarray:
    """nsteps of the 6-D step (Sec. 3.2): x1, x2, x3 sweeps per k-point.

    cubes: full field [k3][k2][k1][x3][x2][x1] (kidx None) or an array of cubes
    [n][x3][x2][x1] whose k-points are kidx[n] = (i1, i2, i3).  slopes: per axis
    (slope_lo, slope_hi) of closure HERMITE.  Returns a new array."""
    f = np.array(cubes, dtype=np.float64, copy=True, order="C")
    nx_a = np.ascontiguousarray(nx, dtype=np.int32)
    nk_a = np.ascontiguousarray(nk, dtype=np.int32)
    M_a = np.ascontiguousarray(M, dtype=np.int32)
    cube = int(nx_a[0]) * int(nx_a[1]) * int(nx_a[2])
    if f.size % cube:
        raise ValueError("field size is not a multiple of the x-cube")
    nkp = f.size // cube
    if kidx is None:
        kp = None
        if nkp != int(nk_a[0]) * int(nk_a[1]) * int(nk_a[2]):
            raise ValueError("full-field call needs nk1*nk2*nk3 cubes")
    else:
        kp = np.ascontiguousarray(kidx, dtype=np.int32).reshape(-1, 3)
        if kp.shape[0] != nkp:
            raise ValueError("kidx length does not match the number of cubes")
    sl = np.zeros((3, 2)) if slopes is None else np.asarray(slopes, dtype=np.float64).reshape(3, 2)
    lo, hi = np.ascontiguousarray(sl[:, 0]), np.ascontiguousarray(sl[:, 1])
    rc = _load().chasm_oracle_advect6d_bc(
        _ip(nx_a), _dp(_f64(hx)), _ip(nk_a), _dp(_f64(klo)), _dp(_f64(hk)), _ip(M_a), int(g), int(closure),
        _dp(lo), _dp(hi), float(dt), int(nsteps), int(nkp), None if kp is None else _ip(kp), _dp(f), int(nthreads))
    _check(rc, "advect6d")
    return f


def reduce(f: np.ndarray, nx, xlo, hx, nk, klo, hk, nb: int = 1) -> np.ndarray:
    """FP64 diagnostics (Sec. 5): [mass, L2^2, <x1>,<x2>,<x3>,<k1>,<k2>,<k3> sums] times cell volume."""
    f = _f64(f)
    out = np.zeros(8)
    nx_a = np.ascontiguousarray(nx, dtype=np.int32)
    nk_a = np.ascontiguousarray(nk, dtype=np.int32)
    _check(_load().chasm_oracle_reduce(_ip(nx_a), _dp(_f64(xlo)), _dp(_f64(hx)), _ip(nk_a), _dp(_f64(klo)),
                                       _dp(_f64(hk)), int(nb), _dp(f), _dp(out)), "reduce")
    return out


def separable_factors(grid, pk, M, g: int, dt: float, nsteps: int, closure: int = PMBC):
    """Advance each packet's 1-D factors with the oracle's line operator.

    On separable data the 6-D step is the tensor product of the three line operators
    (eqs. 3.11-3.12), so after nsteps the field is
    sum_p coef[p] prod_d U[p][d][k_d, x_d] with U[p][d][i] = gk(k_i) * L(alpha_d(k_i))^nsteps gx.
    Returns (coef, U) with U[p][d] of shape (nk_d, nx_d)."""
    from paper_2205_02380_amd import inputs as _inputs
    coef, gx, gk = _inputs.packet_factors(grid, pk)
    hx = grid.hx
    U = []
    for p in range(pk.n):
        Up = []
        for d in range(3):
            N = grid.nx[d]
            c = stencils(N, M[d], g, hx[d], closure)
            kax = grid.k_axis(d)
            rows = np.empty((grid.nk[d], N))
            for i, k in enumerate(kax):
                f = gx[p][d].copy()
                for _ in range(nsteps):
                    f = line(N, M[d], g, hx[d], k * dt / hx[d], f, closure=closure, c=c)
                rows[i] = gk[p][d][i] * f
            Up.append(rows)
        U.append(Up)
    return coef, U


def separable_reference(grid, pk, M, g: int, dt: float, nsteps: int, closure: int = PMBC) -> np.ndarray:
    """Full field of ``separable_factors`` as a numpy array [k3][k2][k1][x3][x2][x1]."""
    coef, U = separable_factors(grid, pk, M, g, dt, nsteps, closure)
    out = np.zeros(grid.shape())
    for p in range(len(coef)):
        a1, a2, a3 = U[p]
        out += coef[p] * (a3[:, None, None, :, None, None] * a2[None, :, None, None, :, None]
                          * a1[None, None, :, None, None, :])
    return out

"""Host build of the HIP path's line algebra (chasm_line.hpp + chasm_tables.cpp), used
only by the CPU tests to compare the product's arithmetic with the oracle off-GPU."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "linetwin.cpp")
TABLES = os.path.join(ROOT, "paper_2205_02380_amd", "csrc", "chasm_tables.cpp")
LINE = os.path.join(ROOT, "paper_2205_02380_amd", "csrc", "chasm_line.hpp")
LIB = os.path.join(HERE, "liblinetwin.so")

# (N, M, G, closure) compiled into the twin
SHAPES = [(8, 2, 1, 0), (8, 4, 3, 0), (8, 4, 3, 1), (8, 8, 7, 0), (8, 8, 7, 1), (16, 8, 4, 0), (16, 8, 4, 1),
          (16, 8, 15, 0), (16, 5, 6, 0), (16, 5, 6, 1), (24, 8, 6, 0), (24, 8, 6, 1), (32, 8, 6, 0), (32, 8, 6, 1),
          (48, 16, 8, 0), (48, 16, 8, 1), (64, 16, 8, 0), (64, 16, 8, 1), (61, 15, 8, 0), (61, 15, 8, 1),
          (8, 4, 3, 2), (16, 8, 4, 2), (16, 8, 15, 2), (32, 8, 6, 2), (61, 15, 8, 2)]


def build() -> str:
    cmd = ["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", SRC, TABLES, "-o", LIB]
    subprocess.run(cmd, check=True, capture_output=True)
    return LIB


_lib = None


def load():
    global _lib
    if _lib is None:
        # CHASM_LINETWIN_LIB: a build of the same sources made elsewhere (the sanitizer run)
        path = os.environ.get("CHASM_LINETWIN_LIB")
        if not path:
            path = LIB
            newest = max(os.path.getmtime(p) for p in (SRC, TABLES, LINE))
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
                build()
        L = ctypes.CDLL(path)
        pd = ctypes.POINTER(ctypes.c_double)
        L.twin_line.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double] * 3 + [pd, pd]
        L.twin_rows.argtypes = [ctypes.c_int] * 4 + [pd]
        L.twin_host_rows.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, pd]
        _lib = L
    return _lib


def line(fp64: bool, N, M, G, CL, h, alpha, phi) -> np.ndarray:
    """One sweep of one line (ghost width G, closure CL) through the product's line
    routine and shift tables: alpha = k dt / h with k = alpha h, dt = 1."""
    out = np.zeros(N)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    pd = ctypes.POINTER(ctypes.c_double)
    rc = load().twin_line(int(fp64), N, M, G, CL, h, alpha * h, 1.0, phi.ctypes.data_as(pd), out.ctypes.data_as(pd))
    if rc != 0:
        raise ValueError(f"twin_line rc={rc}")
    return out


def rows(N, M, G, CL, h=None) -> np.ndarray:
    """Interface rows times h: the kernels' compile-time constants (h None) or the host
    FP64 table builder's rows for spacing h (divided back to rows times h)."""
    P = (N - 1 + M - 1) // M
    out = np.zeros((P + 1, 2 * G + 1))
    pd = ctypes.POINTER(ctypes.c_double)
    if h is None:
        rc = load().twin_rows(N, M, G, CL, out.ctypes.data_as(pd))
    else:
        rc = load().twin_host_rows(N, M, G, CL, float(h), out.ctypes.data_as(pd))
        out *= h
    if rc != 0:
        raise ValueError(f"rows rc={rc}")
    return out

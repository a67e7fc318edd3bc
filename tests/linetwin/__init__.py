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

SHAPES = [(8, 2, 7), (8, 4, 7), (16, 8, 8), (16, 8, 15), (16, 5, 8), (24, 8, 8), (32, 8, 8), (48, 16, 8),
          (64, 16, 8), (61, 15, 8)]


def build() -> str:
    cmd = ["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", SRC, TABLES, "-o", LIB]
    subprocess.run(cmd, check=True, capture_output=True)
    return LIB


_lib = None


def load():
    global _lib
    if _lib is None:
        newest = max(os.path.getmtime(p) for p in (SRC, TABLES, LINE))
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
            build()
        L = ctypes.CDLL(LIB)
        pd = ctypes.POINTER(ctypes.c_double)
        L.twin_line.argtypes = [ctypes.c_int] * 5 + [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                     ctypes.c_double, ctypes.c_double, ctypes.c_int, pd, pd]
        _lib = L
    return _lib


def line(fp64: bool, N, M, G, g, h, closure, alpha, phi) -> np.ndarray:
    """One sweep of one line through the product's tables and line routine."""
    out = np.zeros(N)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    pd = ctypes.POINTER(ctypes.c_double)
    rc = load().twin_line(int(fp64), N, M, G, g, h, closure, 1, alpha * h, 1.0, 1.0, 0, phi.ctypes.data_as(pd),
                          out.ctypes.data_as(pd))
    if rc != 0:
        raise ValueError(f"twin_line rc={rc}")
    return out

"""Build ``libchasm.so`` (gfx950 HIP kernels + C ABI) in-tree with hipcc.

Each .hip unit is compiled separately (in parallel), then linked into one shared
library next to this file.  Run as ``python -m paper_2205_02380_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libchasm.so")
ARCH = "gfx950"

# Packed-FP32 instructions are disabled for all device code.
HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    units = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    return [os.path.join(CSRC, f) for f in units] + [os.path.join(CSRC, "chasm_tables.cpp")]


def _deps(src: str, seen=None) -> set:
    """The source and every local header it includes, transitively."""
    import re
    seen = seen if seen is not None else set()
    if src in seen or not os.path.exists(src):
        return seen
    seen.add(src)
    with open(src) as fh:
        for inc in re.findall(r'#include\s+"([^"]+)"', fh.read()):
            _deps(os.path.normpath(os.path.join(os.path.dirname(src), inc)), seen)
    return seen


def _stale(src: str) -> bool:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(src))


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-c"] + HIPFLAGS + [src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return obj


def build(jobs: int | None = None, verbose: bool = True, incremental: bool = False) -> str:
    """Compile every unit (or, when incremental, only units whose source or local
    headers are newer than their object) and link the library."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if _stale(s)] if incremental else srcs
    jobs = jobs or min(max(len(todo), 1), max(1, min(16, os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(OBJ, os.path.basename(s) + ".o") for s in srcs]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} units ({len(todo)} compiled)")
    return LIB


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--incremental"]
    build(int(args[0]) if args else None, incremental="--incremental" in sys.argv)

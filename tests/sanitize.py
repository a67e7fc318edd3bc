"""CPU sanitizer run: the host C/C++ that the CPU tests execute -- the oracle
(oracle/chasm_oracle.c), the product's FP64 table builder (chasm_tables.cpp) and its
line routine compiled for the host (tests/linetwin) -- built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc/g++, every finding fatal), then the whole
``-m "not gpu"`` suite run against those builds.

    python -m tests.sanitize            # build (cached by source time) and run
    python -m tests.sanitize --build    # build only

The builds go to tests/_san/ (not tracked).  Python itself is not instrumented, so the
ASan runtime is preloaded and leak checking is off (the interpreter's own allocations
at exit are not findings).  No GPU code is involved: the HIP library is only loaded by
the host tests, uninstrumented.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_san")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

ORACLE_SRC = os.path.join(ROOT, "oracle", "chasm_oracle.c")
TWIN_SRC = [os.path.join(HERE, "linetwin", "linetwin.cpp"),
            os.path.join(ROOT, "paper_2205_02380_amd", "csrc", "chasm_tables.cpp")]
TWIN_DEPS = TWIN_SRC + [os.path.join(ROOT, "paper_2205_02380_amd", "csrc", n)
                        for n in ("chasm_line.hpp", "chasm_tables.hpp")]
ORACLE_LIB = os.path.join(OUT, "libchasm_oracle.so")
TWIN_LIB = os.path.join(OUT, "liblinetwin.so")


def _stale(lib, deps):
    return not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(d) for d in deps)


def build():
    os.makedirs(OUT, exist_ok=True)
    if _stale(ORACLE_LIB, [ORACLE_SRC]):
        print("building the oracle with ASan + UBSan", flush=True)
        subprocess.run(["gcc", "-std=c11", "-fopenmp", "-fPIC", "-shared"] + SAN + [ORACLE_SRC, "-o", ORACLE_LIB, "-lm"],
                       check=True)
    if _stale(TWIN_LIB, TWIN_DEPS):
        # host-only compile of the HIP headers' host declarations (no device code)
        print("building the line twin and table builder with ASan + UBSan (a few minutes)", flush=True)
        subprocess.run(["g++", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + SAN
                       + TWIN_SRC + ["-o", TWIN_LIB], check=True)


def runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], check=True, capture_output=True,
                          text=True).stdout.strip()


def main(argv):
    build()
    if "--build" in argv:
        return 0
    env = dict(os.environ)
    env["CHASM_ORACLE_LIB"] = ORACLE_LIB
    env["CHASM_LINETWIN_LIB"] = TWIN_LIB
    env["LD_PRELOAD"] = runtime("libasan.so") + ":" + runtime("libubsan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "tests", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"] + \
        [a for a in argv if a != "--build"]
    print("running:", " ".join(cmd), flush=True)
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))

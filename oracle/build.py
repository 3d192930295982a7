"""Compile the FP64 CPU reference (test infrastructure) into oracle/_build/liboracle.so.

gcc, -O2 with FP contraction off so that every multiply and add is a separate,
correctly rounded FP64 operation in the order the source states; OpenMP splits
work over output rows only, so results do not depend on the thread count.

build_native() makes the timing build of the same source for the machine that
runs it (-O3 -march=native, FP contraction off, no fast-math: the arithmetic and
its order are those of the test build, so results are bitwise the same). It is
compiled on first use on each host, keyed by the host's CPU model, because
-march=native code may not run on another CPU.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emcnn_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


NATIVE_FLAGS = ["-O3", "-march=native", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                "-std=c11", "-Wall"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build_native() -> str:
    """Timing build for this host (see the module docstring); rebuilt when the
    source, the flags or the CPU model differ from the stamp of the last build."""
    os.makedirs(OUT_DIR, exist_ok=True)
    lib = os.path.join(OUT_DIR, "liboracle_native.so")
    stamp = os.path.join(OUT_DIR, "liboracle_native.stamp")
    want = "%s|%s|%s" % (cpu_model(), " ".join(NATIVE_FLAGS), os.path.getmtime(SRC))
    if os.path.exists(lib) and os.path.exists(stamp) and open(stamp).read() == want:
        return lib
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc"] + NATIVE_FLAGS + ["-o", tmp, SRC, "-lm"])
    os.replace(tmp, lib)
    with open(stamp, "w") as f:
        f.write(want)
    return lib


if __name__ == "__main__":
    print(build())

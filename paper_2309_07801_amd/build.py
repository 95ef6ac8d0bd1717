"""Build the gfx950 HIP library libcglbm.so in-tree with hipcc.

The kernels' launch-geometry tables sit in translation units of their own
(csrc/tables.hpp), which compile in parallel and are then linked into one
shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
UNITS = ["cglbm.hip", "fused_tab0.hip", "fused_tab1.hip", "fused_tab2.hip", "cpull_tab.hip",
         "d2q9_tab.hip"]
SRC = os.path.join(CSRC, "cglbm.hip")
LIB = os.path.join(HERE, "libcglbm.so")
OBJDIR = os.path.join(HERE, "_build")
DEPS = [os.path.join(CSRC, n) for n in UNITS + ["kernels.hpp", "lattice.hpp", "d2q9.hpp",
                                                 "tables.hpp", "diag.hpp"]] + [
    os.path.join(ROOT, "include", "cglbm.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # contract a*b+c only inside one source expression, so that the same
    # arithmetic rounds the same way in every kernel it is inlined into
    "-ffp-contract=on",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(n or (os.cpu_count() or 4), 16, len(UNITS)))


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    cmds, objs = [], []
    for u in UNITS:
        obj = os.path.join(OBJDIR, os.path.splitext(u)[0] + ".o")
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + inc + ["-c", "-o", obj, os.path.join(CSRC, u)])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        return subprocess.run(cmd).returncode

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        rcs = list(ex.map(run, cmds))
    if any(rcs):
        raise subprocess.CalledProcessError(max(rcs), "hipcc -c")
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), file=sys.stderr)
    subprocess.check_call(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

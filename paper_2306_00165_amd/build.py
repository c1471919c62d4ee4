"""Build libpcfv.so for gfx950 in-tree (hipcc cross-compiles without a GPU).

Every source is compiled to an object of its own in parallel (the kernel
sources dominate the time), then the objects are linked into the library."""

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_DIR = os.path.join(HERE, "_lib")
OBJ_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(LIB_DIR, "libpcfv.so")
SOURCES = ["csrc/kernels.hip", "csrc/learned.hip", "csrc/capi.cpp", "csrc/capi_learned.cpp", "csrc/tables.cpp",
           "csrc/dmd.cpp", "csrc/eigsym.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def _run(cmd):
    res = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose=False, jobs=None):
    """Compile every source into paper_2306_00165_amd/_lib/libpcfv.so."""
    os.makedirs(LIB_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(OBJ_DIR, os.path.basename(s) + ".o")
        objs.append(o)
        cmds.append([HIPCC] + FLAGS + ["-c", os.path.join(HERE, s), "-o", o])
    if verbose:
        for c in cmds:
            print(" ".join(c))
    with ThreadPoolExecutor(max_workers=jobs or min(len(cmds), os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

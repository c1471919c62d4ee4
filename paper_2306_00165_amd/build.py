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


def _deps(path, seen=None):
    """The file and every local header it includes, recursively."""
    import re
    seen = set() if seen is None else seen
    path = os.path.normpath(path)
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    with open(path) as f:
        for inc in re.findall(r'^\s*#include\s+"([^"]+)"', f.read(), re.M):
            _deps(os.path.join(os.path.dirname(path), inc), seen)
    return seen


def build(verbose=False, jobs=None, incremental=False):
    """Compile every source into paper_2306_00165_amd/_lib/libpcfv.so.  With
    incremental, objects newer than their source and the headers it includes
    are kept."""
    os.makedirs(LIB_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(OBJ_DIR, os.path.basename(s) + ".o")
        objs.append(o)
        src = os.path.join(HERE, s)
        if (incremental and os.path.exists(o) and
                os.path.getmtime(o) > max(os.path.getmtime(d) for d in _deps(src))):
            continue
        cmds.append([HIPCC] + FLAGS + ["-c", src, "-o", o])
    if verbose:
        for c in cmds:
            print(" ".join(c))
    with ThreadPoolExecutor(max_workers=jobs or max(1, min(len(cmds), os.cpu_count() or 1))) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, incremental="--incremental" in sys.argv))

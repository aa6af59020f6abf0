"""Build of the library's shared object (libbeagle.so) for gfx950 with hipcc.

Every HIP source is compiled for gfx950 only and linked, with the host
C-ABI layer, into one shared library placed next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbeagle.so")
SOURCES = ["api.cpp", "batch.cpp", "tune.cpp", "prepare.hip", "eval.hip", "gen.hip", "grad.hip"]
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # no packed-FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast",
    # the interpreter's dispatch branches on a wave-uniform value: leave such
    # regions unstructurized (fewer scalar flag operations per token)
    "-mllvm", "-structurizecfg-skip-uniform-regions",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# per-source flags
SOURCE_FLAGS = {
    # the adjoint handlers each end in a tape write; sinking those writes into
    # one shared block turns every stack slot into a phi (register copies on
    # every word)
    "grad.hip": ["-mllvm", "-simplifycfg-sink-common=false"],
}


def _compile(src: str, build_dir: str = BUILD, defines=(), extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + FLAGS + SOURCE_FLAGS.get(src, []) + list(extra) + [f"-D{d}" for d in defines] + \
        ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=(), extra=()) -> str:
    """Compile and link; ``out`` and ``defines`` (NAME=VALUE) select a
    variant build (tile parameters) placed elsewhere."""
    build_dir = BUILD if out == LIB else os.path.splitext(out)[0] + "_build"
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, defines, extra), SOURCES))
    LIBOUT = out
    tmp = LIBOUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIBOUT)
    if verbose:
        print(f"built {LIBOUT}")
    return LIBOUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

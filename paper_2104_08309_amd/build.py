"""Build libpft.so (HIP, gfx950) in-tree: ``python -m paper_2104_08309_amd.build``.

Compiles every source under ``csrc/`` with hipcc for gfx950 and links them
into ``paper_2104_08309_amd/libpft.so`` next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpft.so")

SOURCES = ["api.cpp", "prologue.hip", "fwd3d.hip", "bwd3d.hip", "fwd2d.hip", "batch.hip", "qorder.hip", "orient.hip",
           "fwdpoly.hip", "dq3d.hip", "loss.hip", "noalloc.hip"]

ARCH = os.environ.get("PFT_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay disabled: the compiler would otherwise form them from scalar float code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiplies and adds fuse only within one source expression: with free fusion across statements the
    # unrolled copies of a loop over a thread's Q points can round differently, and a Q's value would
    # depend on which slot of which thread evaluates it
    "-ffp-contract=on",
    "-I", INCLUDE, "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


# Per-source code generation: the batched FP32C forward's face loop is scheduled for instruction-level
# parallelism (measured faster than the default scheduler, with the same registers and bitwise-identical
# results). The single-mesh forward (fwd3d.hip) keeps the default scheduler: at 2 Q per thread it is
# faster there for both face orders, and the ILP scheduler spilled registers.
FILE_FLAGS = {
    "batch.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libpft)")


def _compile(src: str, hipcc: str, verbose: bool, build_dir: str, defines, src_dir: str) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    flags = [f if f != CSRC else src_dir for f in COMMON]
    cmd = [hipcc] + lang + flags + FILE_FLAGS.get(src, []) + [f"-D{d}" for d in defines] + \
        ["-c", os.path.join(src_dir, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8, out: str = LIB, defines=(), build_dir: str = BUILD,
          src_dir: str = CSRC) -> str:
    """Compile all sources and link the library (default: libpft.so in the package); returns its path.

    ``defines`` are extra preprocessor definitions (tuning constants such as PFT_QPT=2).
    """
    hipcc = _hipcc()
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc, verbose, build_dir, defines, src_dir), SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


UBENCH_SRC = os.path.join(HERE, "ubench", "valu_rates.hip")
UBENCH_BIN = os.path.join(HERE, "ubench", "valu_rates")


def build_ubench(verbose: bool = False, out: str = UBENCH_BIN) -> str:
    """Compile the vector-ALU issue-rate microbenchmark (ubench/valu_rates.hip) with the library's
    code-generation flags into a standalone executable; returns its path."""
    hipcc = _hipcc()
    flags = [f for f in COMMON if f not in ("-fPIC", "-I", INCLUDE, CSRC)]
    tmp = out + ".tmp"
    cmd = [hipcc, "-x", "hip"] + flags + [UBENCH_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {UBENCH_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_ubench(verbose="-v" in sys.argv))

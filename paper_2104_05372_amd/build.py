"""Builds libdexmi.so (HIP kernels + C ABI) for gfx950, in-tree.

    python -m paper_2104_05372_amd.build [--jobs N] [--verbose]

Every source is compiled with hipcc for gfx950 only; the precision-specific
GMM matrix-core file is compiled once per operand precision. Objects go to
paper_2104_05372_amd/_build/, the library to paper_2104_05372_amd/libdexmi.so.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdexmi.so")
ARCH = "gfx950"

# (source, extra defines, object name)
UNITS = [
    ("abi.cpp", [], "abi.o"),
    ("gmm.hip", [], "gmm.o"),
    ("gmm_mfma_inst.hip", ["-DDEX_PREC=0"], "gmm_mfma_f32.o"),
    ("gmm_mfma_inst.hip", ["-DDEX_PREC=1"], "gmm_mfma_bf16.o"),
    ("gmm_mfma_inst.hip", ["-DDEX_PREC=2"], "gmm_mfma_bf16x3.o"),
    ("gmm_batched.hip", [], "gmm_batched.o"),
    ("scatter.hip", [], "scatter.o"),
    ("stencil.hip", [], "stencil.o"),
    ("reduce.hip", [], "reduce.o"),
]

# -packed-fp32-ops: no packed FP32 instructions are generated (they are kept
# out of every kernel on purpose). The host pass warns that it does not know
# the feature; that warning is harmless.
# -amdgpu-mfma-vgpr-form: matrix-core results stay in ordinary VGPRs, so the
# epilogues read them without accumulator-register copies and the kernels need
# about half the registers (more waves per SIMD).
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I", os.path.join(os.path.dirname(PKG), "include"),
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(unit, verbose):
    src, defs, obj = unit
    cmd = [hipcc(), *CFLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} {' '.join(defs)} failed:\n{err}")
    if verbose and err.strip():
        print(err)
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every unit and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)), 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[os.path.join(BUILD, o) for o in objs]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose))


if __name__ == "__main__":
    sys.exit(main())

"""Builds the HIP shared libraries in-tree for gfx950.

* ``paper_2007_08056_amd/libsymtensor.so`` -- the contraction library (C ABI
  of include/symtensor.h).
* ``synth/libsynthgen.so`` -- the GPU twin of the seeded input generator.
* ``synth/libphilox_host.so`` -- its host twin in C (test inputs and samples).

Usage: ``python paper_2007_08056_amd/build.py`` (always recompiles).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ARCH = os.environ.get("SYMT_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 ops are disabled for all device code.  MFMA accumulators live in
# VGPRs (gfx950 MFMAs read and write C/D there): otherwise loop-carried
# accumulators are copied through AGPRs around every K-step, and reading an
# MFMA result back drains the matrix pipe each time.
COMMON = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-amdgpu-mfma-vgpr-form"]

LIB_SOURCES = ["plan.cpp", "symtensor.cpp", "xform.hip", "gemm.hip", "scratch.hip", "gemm_bf16x3.hip", "gemm_rows.hip", "gemm_tallk.hip"]
# The wide split-bf16 tiles keep their 256 accumulators in AGPRs: built without
# the VGPR-form flag.
NO_VGPR_FORM = {"gemm_bf16x3.hip"}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out, flush=True)


def build_symtensor(verbose=False) -> str:
    csrc = os.path.join(HERE, "csrc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    objs = []
    cmds = []
    for src in LIB_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        flags = [f for f in COMMON if f not in ("-mllvm", "-amdgpu-mfma-vgpr-form")] if src in NO_VGPR_FORM else COMMON
        cmds.append([HIPCC] + flags + inc + lang + ["-c", os.path.join(csrc, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    out = os.path.join(HERE, "libsymtensor.so")
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, out)
    return out


def build_synth(verbose=False) -> str:
    src = os.path.join(ROOT, "synth", "csrc", "synth_gen.hip")
    out = os.path.join(ROOT, "synth", "libsynthgen.so")
    tmp = out + ".tmp"
    _run([HIPCC] + COMMON + ["-ffp-contract=off", "-shared", "-x", "hip", src, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build_synth_host(verbose=False) -> str:
    src = os.path.join(ROOT, "synth", "csrc", "philox_host.c")
    out = os.path.join(ROOT, "synth", "libphilox_host.so")
    tmp = out + ".tmp"
    _run([os.environ.get("CC", "gcc"), "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", src,
          "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


def build_all(verbose=False):
    return build_symtensor(verbose), build_synth(verbose), build_synth_host(verbose)


if __name__ == "__main__":
    for p in build_all(verbose="-v" in sys.argv):
        print("built", p)

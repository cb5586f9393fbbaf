"""Builds the gfx950 shared library libbltc.so in-tree.

    python -m paper_2003_01836_amd.build

Host planning code is compiled by g++ without floating-point contraction (its
geometric decisions follow their formulas operation by operation); the HIP
sources are compiled by hipcc for gfx950 only.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libbltc.so")
MICROBENCH = os.path.join(PKG, "microbench")

ARCH = "gfx950"
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             # no packed-FP32 instructions anywhere in device code
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + INCLUDE, "-I" + CSRC, "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
              "-I" + INCLUDE, "-I" + CSRC, "-Wall"]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run_all(cmds):
    procs = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for c in cmds]
    failed = []
    for c, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass of hipcc does not know the packed-FP32 feature; that note is harmless
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append((c, "\n".join(lines)))
        elif any(ln.strip() for ln in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + t for c, t in failed)
        raise RuntimeError("build failed:\n" + msg)


def build(verbose: bool = False, defines=(), lib_path: str = LIB, build_dir: str = BUILD) -> str:
    """Compiles libbltc.so; `defines` are extra -D flags for the HIP sources."""
    os.makedirs(build_dir, exist_ok=True)
    hipcc = _hipcc()
    hip_flags = HIP_FLAGS + ["-D" + d for d in defines]
    objs = {
        "planner": os.path.join(build_dir, "planner.o"),
        "kernels": os.path.join(build_dir, "kernels.o"),
        "mixed": os.path.join(build_dir, "kernels_mixed.o"),
        "mrhs": os.path.join(build_dir, "kernels_mrhs.o"),
        "upward": os.path.join(build_dir, "kernels_upward.o"),
        "capi": os.path.join(build_dir, "capi.o"),
        "batch": os.path.join(build_dir, "batch.o"),
        "autotune": os.path.join(build_dir, "autotune.o"),
        "setup": os.path.join(build_dir, "setup_gpu.o"),
        "cp": os.path.join(build_dir, "cp.o"),
        "cc": os.path.join(build_dir, "cc.o"),
        "kernels_cp": os.path.join(build_dir, "kernels_cp.o"),
        "kernels_hermite": os.path.join(build_dir, "kernels_hermite.o"),
        "kernels_sym": os.path.join(build_dir, "kernels_sym.o"),
        "kernels_split": os.path.join(build_dir, "kernels_split.o"),
        "noalloc": os.path.join(build_dir, "noalloc.o"),
    }
    cmds = [
        ["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, "planner.cpp"), "-o", objs["planner"]],
        [hipcc] + hip_flags + ["-c", os.path.join(CSRC, "kernels.hip"), "-o", objs["kernels"]],
        [hipcc] + hip_flags + ["-c", os.path.join(CSRC, "kernels_mixed.hip"), "-o", objs["mixed"]],
        # MFMA accumulators stay in VGPRs (no AGPR round trip around every step)
        [hipcc] + hip_flags + ["-mllvm", "-amdgpu-mfma-vgpr-form",
                               "-c", os.path.join(CSRC, "kernels_mrhs.hip"), "-o", objs["mrhs"]],
        [hipcc] + hip_flags + ["-mllvm", "-amdgpu-mfma-vgpr-form",
                               "-c", os.path.join(CSRC, "kernels_upward.hip"), "-o", objs["upward"]],
        [hipcc] + hip_flags + ["-x", "hip", "-c", os.path.join(CSRC, "capi.cpp"), "-o", objs["capi"]],
        [hipcc] + hip_flags + ["-x", "hip", "-c", os.path.join(CSRC, "batch.cpp"), "-o", objs["batch"]],
        [hipcc] + hip_flags + ["-x", "hip", "-c", os.path.join(CSRC, "autotune.cpp"), "-o", objs["autotune"]],
        # geometric decisions (MAC) follow their formulas operation by operation
        [hipcc] + hip_flags + ["-ffp-contract=off", "-c", os.path.join(CSRC, "setup_gpu.hip"), "-o", objs["setup"]],
        [hipcc] + hip_flags + ["-x", "hip", "-c", os.path.join(CSRC, "cp.cpp"), "-o", objs["cp"]],
        [hipcc] + hip_flags + ["-x", "hip", "-c", os.path.join(CSRC, "cc.cpp"), "-o", objs["cc"]],
        [hipcc] + hip_flags + ["-c", os.path.join(CSRC, "kernels_cp.hip"), "-o", objs["kernels_cp"]],
        [hipcc] + hip_flags + ["-c", os.path.join(CSRC, "kernels_hermite.hip"), "-o",
                               objs["kernels_hermite"]],
        [hipcc] + hip_flags + ["-c", os.path.join(CSRC, "kernels_sym.hip"), "-o",
                               objs["kernels_sym"]],
        [hipcc] + hip_flags + ["-c", os.path.join(CSRC, "kernels_split.hip"), "-o",
                               objs["kernels_split"]],
        [hipcc] + hip_flags + ["-c", os.path.join(CSRC, "noalloc.hip"), "-o", objs["noalloc"]],
    ]
    if verbose:
        for c in cmds:
            print(" ".join(c))
    _run_all(cmds)
    tmp = lib_path + ".tmp"
    link = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + list(objs.values()) + ["-lpthread"]
    _run_all([link])
    os.replace(tmp, lib_path)
    build_microbench()
    return lib_path


def build_microbench(exe_path: str = MICROBENCH) -> str:
    """Compiles the instruction-cost probes (csrc/microbench.hip) into a standalone
    program; bench.py's issue-rate model takes its constants from their output."""
    tmp = exe_path + ".tmp"
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-o", tmp, os.path.join(CSRC, "microbench.hip")]
    _run_all([cmd])
    os.replace(tmp, exe_path)
    return exe_path


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the HIP library (libtddftb.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtddftb.so")
SOURCES = ["gemm_f64.hip", "gemm_split_bf16.hip", "kernels.hip", "batch_kernels.hip", "tddftb.hip",
           "batch.hip", "spectra.hip", "ehrenfest_kernels.hip", "plus_u_kernels.hip",
           "noalloc.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


LIB_SANITIZED = os.path.join(PKG, "libtddftb_sanitized.so")
# host code only (the device code is built as usual): AddressSanitizer and
# UndefinedBehaviorSanitizer, against the shared ASan runtime, which the
# loading process preloads
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-shared-libasan"]


def sanitizer_runtime() -> str:
    """Path of the shared ASan runtime of ROCm's clang (to preload)."""
    import glob
    found = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(hipcc())), "lib", "llvm",
                                          "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    if not found:
        raise RuntimeError("no shared ASan runtime found next to hipcc")
    return found[-1]


def command(out: str = LIB, sanitize: bool = False) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            *(SANITIZE if sanitize else []),
            "-Wall", "-Wno-unused-function",
            # no packed-FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # matrix-core accumulators in ordinary VGPRs: avoids AGPR<->VGPR
            # copies of the accumulators around the K loop (gfx950 allows both)
            "-mllvm", "-amdgpu-mfma-vgpr-form",
            "-I", INCLUDE, *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def build(verbose: bool = True, sanitize: bool = False) -> str:
    """Builds libtddftb.so, or with `sanitize` libtddftb_sanitized.so (host
    code under ASan and UBSan, for the CPU tests of the C ABI)."""
    lib = LIB_SANITIZED if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = command(tmp, sanitize)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build()

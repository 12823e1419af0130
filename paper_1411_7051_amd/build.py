"""Build the HIP library ``liblbk.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbk.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
SOURCES = ["lbk_kernels.hip", "lbk_adjoint.hip", "lbk_api.hip", "lbk_batch.hip",
           "lbk3_kernels.hip", "lbk3_api.hip", "lbk_noalloc.hip"]
HEADERS = ["lbk_device.h", "lbk_kernels.h", "lbk_adjoint.h", "lbk_host.h", "lbk3_kernels.h"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a*b+c only within one source expression: the node update then
    # rounds identically in every kernel that inlines it (single lattice,
    # batched tile list, adjoint recompute), whatever the control flow around
    "-ffp-contract=on",
]


def libs() -> list:
    """roctx (ranges around the host-side phases: stepping, gradients, graph
    replays), found at run time through the ROCm library directory."""
    lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    return [f"-L{lib}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{lib}"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source into ``liblbk.so`` (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", INCLUDE, *extra, "-o", tmp, *srcs, *libs()]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])

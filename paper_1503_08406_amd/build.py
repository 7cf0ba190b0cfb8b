"""Build the HIP library libdmrt.so for gfx950 (in-tree, next to this file)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdmrt.so")
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("dmrt_step.hip", "dmrt_step2.hip", "dmrt_batch.hip", "dmrt_adjoint.hip", "dmrt_kernels.hip", "dmrt_api.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are disabled: hipcc emits them from plain
    # float code and some of their forms are unreliable on this hardware
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused within one source expression only: whether
    # two statements fuse would otherwise depend on the surrounding code,
    # and the one- and two-step kernels (and the batched ones) must round
    # every node's arithmetic the same way
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False, extra=()):
    """Compile every source into libdmrt.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])

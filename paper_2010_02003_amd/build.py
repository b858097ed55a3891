"""Build the HIP library ``libdg2.so`` for gfx950 in the package directory.

    python -m paper_2010_02003_amd.build

Compiles the kernels and the C-ABI runtime in one hipcc invocation.  Packed
FP32 instruction forms are disabled for the device code, and multiply-adds
are contracted only within one expression.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdg2.so")
SOURCES = ["dg2_kernels.hip", "dg2_api.hip", "dg2_adjoint.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def flags():
    # -ffp-contract=on: a*b+c is fused only within one source expression, so
    # every inlined copy of a formula rounds alike and results do not depend
    # on the launch shape (hipcc's default lets the backend fuse across
    # statements differently in different copies).
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, csrc: str = CSRC, out: str = LIB, extra=()) -> str:
    srcs = [os.path.join(csrc, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [HIPCC] + flags() + ["-I", csrc] + list(extra) + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

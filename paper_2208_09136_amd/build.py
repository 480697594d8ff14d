"""Build the gfx950 shared library librqa.so in place (hipcc cross-compiles
without a GPU).

Flags that matter for the results:
  -ffp-contract=off                   no fused multiply-add anywhere, so keys
                                      are the binary32 values of the plain
                                      left-to-right arithmetic
  -fno-gpu-flush-denormals-to-zero    keep binary32 denormals
  -target-feature -packed-fp32-ops    no packed FP32 instructions
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librqa.so")
SOURCES = ["kernels.hip", "mlp.hip", "capi.hip"]
ARCH = os.environ.get("RQA_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def build(verbose=False, out=None, defines=()):
    """Compile librqa.so (or `out`); `defines` are extra -D options."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + ["-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)

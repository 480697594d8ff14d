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
SOURCES = ["kernels.hip", "mlp.hip", "probe.hip", "capi.hip"]
ARCH = os.environ.get("RQA_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def build(verbose=False, out=None, defines=()):
    """Compile librqa.so (or `out`); `defines` are extra -D options.  The
    sources compile to objects in parallel (no device code crosses a source
    file: every kernel is launched from its own file), then link."""
    lib = out or LIB
    tmp = lib + ".tmp"
    objdir = os.path.join(os.path.dirname(lib), "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    defs = ["-D" + d for d in defines]
    procs, objs = [], []
    for name in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(name)[0] + ".o")
        cmd = [HIPCC] + compile_flags + defs + ["-c", "-o", obj, os.path.join(CSRC, name)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)

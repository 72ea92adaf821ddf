"""Compile librmc.so (HIP kernels + host runtime) for gfx950, in-tree.

Packed-FP32 instruction selection is disabled for all device code
(-target-feature -packed-fp32-ops).
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "librmc.so")
SOURCES = ["csrc/rmc_kernels.hip", "csrc/rmc_api.cpp"]


def hipcc_cmd(out=LIB, defines=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return [hipcc, "--offload-arch=gfx950", "-mcode-object-version=5", "-O3", "-std=c++17", "-fPIC",
            "-shared"] + list(defines) + [
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
            "-o", out] + [os.path.join(PKG, s) for s in SOURCES]


def build(verbose=False, out=LIB, defines=()):
    tmp = out + ".tmp"
    cmd = hipcc_cmd(tmp, defines)
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    log = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + log)
    if verbose and log.strip():
        print(log)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build the gfx950 HIP library liblbm.so in-tree with hipcc.

Every kernel is compiled for gfx950 only.  Packed FP32 instructions are
disabled for the device code (-packed-fp32-ops); the host pass warns that it
does not know that feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIB_DIR, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm_api.hip"), os.path.join(CSRC, "nn_api.hip"), os.path.join(CSRC, "probe.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: a multiply is fused with an add only inside one source
# expression, never across statements, so the same update rounds the same
# way wherever it is inlined (the single-step and the streaming kernels must
# agree bit for bit).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Wall", "-ffp-contract=on", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False, extra=None) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra or []) + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the HIP library in-tree: paper_1404_1719_amd/lib/libvtxrates.so (gfx950).

Usage: python -m paper_1404_1719_amd.build_lib   (or call build()).
hipcc cross-compiles for gfx950 without a GPU. Packed FP32 instructions are disabled for
the device code (-Xclang -target-feature -Xclang -packed-fp32-ops)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "lib", "libvtxrates.so")
SOURCES = [os.path.join(CSRC, "vtx_kernels.hip"), os.path.join(CSRC, "vtx_newton.hip"),
           os.path.join(CSRC, "vtx_massive.hip"),
           os.path.join(CSRC, "vtx_host.cpp")]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

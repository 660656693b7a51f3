"""Compile libsse.so for gfx950 with hipcc (in-tree, next to this file).

Flags that matter for the numerics:
  -ffp-contract=off                         no fused multiply-add contraction
  -fhip-fp32-correctly-rounded-divide-sqrt  IEEE-rounded binary32 / and sqrt
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                            no packed binary32 instructions
  -munsafe-fp-atomics                       hardware binary64 atomic add
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsse.so")
SOURCES = ["csrc/transport.hip", "csrc/post.hip", "csrc/recon.hip", "csrc/capi.cpp", "csrc/serve.cpp",
           "csrc/recon_api.cpp"]
# throughput microbenchmarks of the device (measurement support, its own library)
PEAKS_LIB = os.path.join(HERE, "libsse_peaks.so")
PEAKS_SOURCES = ["csrc/peaks.hip"]
ARCH = os.environ.get("SSE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
            "-fhip-fp32-correctly-rounded-divide-sqrt", "-munsafe-fp-atomics",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    _link(SOURCES, LIB, verbose)
    _link(PEAKS_SOURCES, PEAKS_LIB, verbose)
    return LIB


def _link(sources, lib, verbose):
    objs = []
    for src in sources:
        path = os.path.join(HERE, src)
        obj = os.path.join(HERE, "csrc", os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + flags() + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

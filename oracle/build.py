"""Build the C oracle (test infrastructure) with gcc.

Two shared libraries come out of the sources (sse_oracle.c, and recon.c,
the reconstruction of the estimation loop, binary64 in both):
  liboracle_f32.so  transport in binary32 (the kernel's precision)
  liboracle_f64.so  transport in binary64
Flags: -O2, no fast-math, no floating-point contraction, SSE arithmetic
(x86-64 default), so every binary32 / binary64 operation is IEEE-rounded.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
VARIANTS = {"f32": "float", "f64": "double"}


def lib_path(variant: str) -> str:
    return os.path.join(HERE, f"liboracle_{variant}.so")


def build(verbose: bool = False) -> None:
    src = os.path.join(HERE, "sse_oracle.c")
    recon = os.path.join(HERE, "recon.c")
    for variant, real in VARIANTS.items():
        out = lib_path(variant)
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wextra", "-Wno-unused-parameter", f"-DORACLE_REAL={real}",
               src, recon, "-o", out + ".tmp", "-lm", "-pthread"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

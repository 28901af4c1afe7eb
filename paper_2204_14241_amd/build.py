"""Build libhmc.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2204_14241_amd.build   (or build_library() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhmc.so")
SOURCES = [os.path.join(CSRC, "hmc.hip")]
DEPS = SOURCES + [os.path.join(CSRC, f) for f in ("kernels.h", "lattice.h", "fft.h", "precond.h", "metric.h", "probe.h", "march.h")] + [
    os.path.join(ROOT, "include", f) for f in ("hmc.h", "hmc_testing.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def source_hash():
    """First 16 hex digits of the SHA-256 of every source and header the library is built from
    (keys the autotuner's on-disk cache to the kernels it timed)."""
    import hashlib
    h = hashlib.sha256()
    for f in DEPS:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build_library(verbose=False):
    """Compile every HIP source into paper_2204_14241_amd/libhmc.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, f'-DHMC_SOURCE_HASH="{source_hash()}"', *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose=True)
    print("built", LIB)
    sys.exit(0)

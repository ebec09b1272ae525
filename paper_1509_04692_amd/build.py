"""Build libhpmc.so for gfx950 in-tree with hipcc.

Flags: binary64 expressions are never contracted into fused multiply-adds
(-ffp-contract=off) so that the FP64 path reproduces its pinned operation
order; packed binary32 instructions are disabled on the device.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB_DIR = os.path.join(PKG, "lib")
LIB_PATH = os.path.join(LIB_DIR, "libhpmc.so")
# the same sources with the per-wave phase clock compiled in (-DHPMC_TRACE)
TRACE_LIB_PATH = os.path.join(LIB_DIR, "libhpmc_trace.so")
SOURCES = ["api.hip", "kernels.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def hipcc_path():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build_library(verbose=True, extra_flags=(), trace=False):
    """Compile every HIP source into lib/libhpmc.so (always recompiles);
    trace=True builds lib/libhpmc_trace.so with the phase clock."""
    os.makedirs(LIB_DIR, exist_ok=True)
    out = TRACE_LIB_PATH if trace else LIB_PATH
    if trace:
        extra_flags = (*extra_flags, "-DHPMC_TRACE")
    tmp = out + ".tmp"
    cmd = [hipcc_path(), *HIPCC_FLAGS, *extra_flags, "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed to build {os.path.basename(out)}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build_library(trace="--trace" in sys.argv)

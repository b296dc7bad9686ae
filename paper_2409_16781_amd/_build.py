"""Build the HIP library in-tree: paper_2409_16781_amd/liblbm355.so (gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm355.so")
SOURCES = [os.path.join(CSRC, n) for n in ("lb_capi.hip", "lb_batch.hip", "lb_d2q9.hip", "lb_kernels.hip")]

# -packed-fp32-ops: no packed FP32 instructions in device code (ordinary FP32
# VALU only).  The host pass reports the feature as unknown; that is harmless.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(out: str = LIB, extra=None, verbose: bool = False) -> str:
    """Compile every HIP source into one shared library (always recompiles)."""
    tmp = out + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra or []) + [
        "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-6000:])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

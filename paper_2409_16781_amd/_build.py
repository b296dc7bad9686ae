"""Build the HIP library in-tree: paper_2409_16781_amd/liblbm355.so (gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm355.so")
SOURCES = [os.path.join(CSRC, n) for n in ("lb_capi.hip", "lb_batch.hip", "lb_d2q9.hip", "lb_kernels.hip",
                                           "lb_batch_kernels.hip", "lb_adjoint_kernels.hip", "lb_aa_kernels.hip",
                                           "lb_d2q9_kernels.hip")]

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


def build(out: str = LIB, extra=None, verbose: bool = False, objdir: str = None) -> str:
    """Compile every HIP source (in parallel, one object each) and link one
    shared library (always recompiles).  extra: more hipcc flags; objdir:
    where the objects go (default paper_2409_16781_amd/_build)."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = objdir or os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = [f for f in HIPCC_FLAGS if f != "-shared"] + list(extra or [])
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc()] + flags + inc + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n" + res.stderr[-6000:])
        return obj

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr[-6000:])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

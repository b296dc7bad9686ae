"""Write tgv512_noise_golden.{json,npz}: FP64 oracle results of the 512^3
Taylor-Green + noise workload.

Workload: D3Q19 BGK, periodic 512 x 512 x 512 sites, Taylor-Green vortex
(u0 = 0.01, k = 2 pi / 512, uniform in z) plus i.i.d. U(+-1e-3) noise on each
velocity component (seed 2), tau = 0.55, no force, 1000 steps.  The paper
names the Taylor-Green vortex among its use cases (Section 3.3); the solver is
Eq. 1-3 in the fused form of Section 3.1.

Stored, after 200 and after 1000 steps:
  * rho and u at 16384 seeded sample sites (npz, float64);
  * whole-field statistics: sum of u_a^2 per component, sum of (rho - 1)^2,
    the amplitude of the initial Taylor-Green mode (the projection of u onto
    it), max |u|, and the conservation totals (mass, momentum).

Calls only the oracle and the input generators.  Needs about 42 GB of host
memory (two FP64 states of 20.4 GB) and about an hour on 8 cores: run it once
with `python tests/golden/make_tgv512_noise_golden.py`.
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2409_16781_amd import inputs  # noqa: E402

OUT_JSON = os.path.join(HERE, "tgv512_noise_golden.json")
OUT_NPZ = os.path.join(HERE, "tgv512_noise_golden.npz")
N = 512
SAMPLES = 16384
SAMPLE_SEED = 11
CHECKPOINTS = (200, 1000)


def sample_sites(n, count, seed):
    """Distinct seeded sites (z, y, x), sorted by linear index."""
    rng = np.random.default_rng(seed)
    lin = np.sort(rng.choice(n ** 3, size=count, replace=False))
    return np.stack([lin // (n * n), (lin // n) % n, lin % n], axis=1).astype(np.int64)


def tgv_mode(n):
    """(ny, nx) shape of the initial mode: (sin kx cos ky, -cos kx sin ky)."""
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=np.float64)
    sx, cx, sy, cy = np.sin(k * x), np.cos(k * x), np.sin(k * x), np.cos(k * x)
    return np.outer(cy, sx), -np.outer(sy, cx)


def field_stats(rho, u):
    """Whole-field statistics of (rho, u); the same definition is evaluated on
    the GPU result by the test."""
    mx, my = tgv_mode(rho.shape[-1])
    proj = float(np.einsum("zyx,yx->", u[0], mx) + np.einsum("zyx,yx->", u[1], my))
    norm = float(rho.shape[0] * ((mx * mx).sum() + (my * my).sum()))
    return {
        "sum_u2": [float(np.einsum("zyx,zyx->", u[a], u[a])) for a in range(3)],
        "sum_drho2": float(np.einsum("zyx,zyx->", rho - 1.0, rho - 1.0)),
        "mode_amplitude": proj / norm,
        "max_abs_u": float(np.abs(u).max()),
    }


def main():
    oracle.build(force=False)
    t0 = time.time()
    cfg = inputs.tgv_noise_box(N, u0=0.01, tau=0.55, steps=1000, noise=1e-3, seed=2)
    sites = sample_sites(N, SAMPLES, SAMPLE_SEED)
    z, y, x = sites[:, 0], sites[:, 1], sites[:, 2]
    S = oracle.init(cfg["shape"], cfg["rho"], cfg["u"])
    init_stats = field_stats(cfg["rho"], cfg["u"])
    del cfg["rho"], cfg["u"]
    meta = {
        "workload": "D3Q19 BGK periodic 512^3 Taylor-Green u0=0.01 k=2pi/512 (uniform in z) "
                    "+ U(+-1e-3) noise on each u component (seed 2, numpy default_rng, C order (3, z, y, x)), "
                    "tau=0.55, F=0",
        "source": "FP64 oracle (oracle/d3q19_oracle.c), written by tests/golden/make_tgv512_noise_golden.py",
        "sample_seed": SAMPLE_SEED,
        "samples": SAMPLES,
        "initial": init_stats,
        "initial_sums": [float(v) for v in oracle.sums(S)],
        "checkpoints": {},
    }
    arrays = {"sites_zyx": sites}
    done = 0
    for n in CHECKPOINTS:
        t1 = time.time()
        oracle.run(S, cfg["tau"], n - done, copy=False)
        done = n
        rho, u = oracle.macros(S)
        st = field_stats(rho, u)
        st["sums"] = [float(v) for v in oracle.sums(S)]
        st["seconds"] = round(time.time() - t1, 1)
        meta["checkpoints"][str(n)] = st
        arrays[f"rho_{n}"] = rho[z, y, x].copy()
        arrays[f"u_{n}"] = u[:, z, y, x].T.copy()
        del rho, u
        print(f"step {n}: {st}", flush=True)
    meta["seconds"] = round(time.time() - t0, 1)
    np.savez_compressed(OUT_NPZ, **arrays)
    with open(OUT_JSON, "w") as f:
        json.dump(meta, f, indent=1)
    print(f"wrote {OUT_JSON} and {OUT_NPZ} in {meta['seconds']} s", flush=True)


if __name__ == "__main__":
    main()

"""Write channel256x128x128_5000.json: FP64 oracle results for the channel workload.

Workload: D3Q19 BGK, 256 x 128 x 128 sites, solid planes y = 0 and y = 127,
periodic in x and z, body force (1e-6, 0, 0), tau = 0.6, rho = 1 + U(+-1e-4)
(seed 1), u = 0, 5000 steps.  Stored: the x-z averaged velocity profile
u_x(y), the macroscopic fields at 512 seeded sample sites, and the
conservation totals of the final state.

Calls only the oracle and the input generators.  Takes minutes (about 21e9
site updates): run it once with `python tests/golden/make_channel_golden.py`.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2409_16781_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "channel256x128x128_5000.json")


def sample_sites(flags, count, seed):
    rng = np.random.default_rng(seed)
    fluid = np.argwhere(flags == 0)
    pick = rng.choice(len(fluid), size=count, replace=False)
    return [tuple(int(v) for v in fluid[k]) for k in sorted(pick)]


def main(steps=5000):
    oracle.build(force=False)
    cfg = inputs.channel(256, 128, 128, tau=0.6, g=1e-6, steps=steps, noise=1e-4, seed=1)
    t0 = time.time()
    S = oracle.init(cfg["shape"], cfg["rho"], cfg["u"], cfg["flags"])
    S = oracle.run(S, cfg["tau"], steps, F=cfg["force"], flags=cfg["flags"])
    rho, u = oracle.macros(S, F=cfg["force"], flags=cfg["flags"])
    sums = oracle.sums(S, cfg["flags"])
    fl = cfg["flags"]
    prof = [float(u[0, :, y, :].mean()) if y not in (0, 127) else 0.0 for y in range(128)]
    sites = sample_sites(fl, 512, 7)
    data = {
        "workload": "D3Q19 BGK channel 256x128x128 (z, y, x) = (128, 128, 256), walls y=0,127, periodic x,z, "
                    "F=(1e-6,0,0), tau=0.6, rho=1+U(+-1e-4) seed 1, u=0",
        "steps": steps,
        "source": "FP64 oracle (oracle/d3q19_oracle.c), written by tests/golden/make_channel_golden.py",
        "seconds": round(time.time() - t0, 1),
        "profile_ux": prof,
        "sites_zyx": sites,
        "rho": [float(rho[s]) for s in sites],
        "u": [[float(u[a][s]) for a in range(3)] for s in sites],
        "sums": [float(v) for v in sums],
    }
    with open(OUT, "w") as f:
        json.dump(data, f)
    print(f"wrote {OUT} in {data['seconds']} s")


if __name__ == "__main__":
    main()

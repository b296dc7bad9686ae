"""Write porous128_grad500.json: FP64 oracle gradient of the outlet mass flux.

Workload: D3Q19 BGK, 128^3 porous channel (walls at y = 0 and 127, random
spheres of radius U[2, 6] to porosity 0.85, seed 4), tau = 0.6, uniform force
(1e-6, 0, 0), at rest initially, 500 steps.  Objective: J = sum of rho u_x over
the fluid sites of the plane x = 127 after 500 steps.  Stored: J, dJ/dF_x
(the derivative with respect to a per-site x-force field, evaluated at a
zero field) at 2048 seeded fluid cells plus 64 outlet cells, and the L2 norm
and sum of dJ/dF_x over all cells.

Calls only the oracle and the input generators (checkpoints every 25 steps).
Takes several minutes: run it once with
`python tests/golden/make_adjoint_golden.py`.
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

OUT = os.path.join(HERE, "porous128_grad500.json")


def main():
    oracle.build(force=False)
    cfg = inputs.porous_channel(128, porosity=0.85, tau=0.6, g=1e-6, seed=4, steps=500, every=50)
    t0 = time.time()
    S0 = oracle.init(cfg["shape"], cfg["rho"], cfg["u"], cfg["flags"])
    J, grad = oracle.grad_outlet_flux(S0, cfg["tau"], cfg["steps"], F=cfg["force"], flags=cfg["flags"],
                                      Fx_field=np.zeros(cfg["shape"]), every=25)
    fl = cfg["flags"]
    rng = np.random.default_rng(41)
    fluid = np.argwhere(fl == 0)
    cells = [tuple(int(v) for v in fluid[k]) for k in sorted(rng.choice(len(fluid), 2048, replace=False))]
    outlet = [tuple(int(v) for v in c) for c in fluid if c[2] == 127]
    cells += [outlet[k] for k in sorted(rng.choice(len(outlet), 64, replace=False))]
    data = {
        "workload": "D3Q19 BGK 128^3 porous channel, walls y=0,127 + spheres r~U[2,6] to porosity 0.85 (seed 4), "
                    "tau=0.6, F=(1e-6,0,0), rest start, 500 steps; J = sum rho u_x at x=127",
        "steps": cfg["steps"],
        "source": "FP64 oracle (oracle/d3q19_oracle.c adjoint), written by tests/golden/make_adjoint_golden.py",
        "seconds": round(time.time() - t0, 1),
        "J": J,
        "cells_zyx": cells,
        "grad": [float(grad[c]) for c in cells],
        "grad_l2": float(np.sqrt((grad * grad).sum())),
        "grad_sum": float(grad.sum()),
    }
    with open(OUT, "w") as f:
        json.dump(data, f)
    print(f"wrote {OUT} in {data['seconds']} s")


if __name__ == "__main__":
    main()

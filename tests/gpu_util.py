"""Helpers shared by the GPU tests: run a workload through the C ABI (via the
binding) and through the oracle, and compare."""
from __future__ import annotations

import os
import sys
from contextlib import contextmanager

import numpy as np

import paper_2409_16781_amd as lbm


def require_gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def say(*a):
    """Name the case on stderr before each GPU step (survives a crash)."""
    print(*a, file=sys.stderr, flush=True)


@contextmanager
def kernel_variant(v):
    """Select the step kernel for lattices created inside the block (0..3 or None)."""
    old = os.environ.get("LB_KERNEL")
    if v is None:
        os.environ.pop("LB_KERNEL", None)
    else:
        os.environ["LB_KERNEL"] = str(v)
    try:
        yield
    finally:
        if old is None:
            os.environ.pop("LB_KERNEL", None)
        else:
            os.environ["LB_KERNEL"] = old


def make_lattice(cfg, codec="f32", variant=None):
    torch = require_gpu()
    nz, ny, nx = cfg["shape"]
    with kernel_variant(variant):
        lat = lbm.Lattice(nx, ny, nz, cfg["tau"], flags=cfg.get("flags"), codec=codec)
    F = cfg.get("force", (0.0, 0.0, 0.0))
    lat.set_force(*F)
    rho = None if cfg.get("rho") is None else torch.from_numpy(np.ascontiguousarray(cfg["rho"], np.float64)).cuda()
    u = None if cfg.get("u") is None else torch.from_numpy(np.ascontiguousarray(cfg["u"], np.float64)).cuda()
    lat.init_eq(rho, u)
    return lat


def gpu_run(cfg, steps, codec="f32", variant=None, same_pass=False):
    """Returns (rho, u) float64 numpy after ``steps`` steps, and the lattice."""
    lat = make_lattice(cfg, codec, variant)
    say(f"[gpu] {cfg.get('name', '?')} {cfg['shape']} codec={codec} variant={lat.info['variant']} steps={steps}")
    if same_pass and steps > 0:
        r, u = lat.step_macros(steps)
    else:
        lat.step(steps)
        r, u = lat.macros()
    lat.sync()
    return r.double().cpu().numpy(), u.double().cpu().numpy(), lat


def oracle_run(cfg, steps):
    import oracle

    S = oracle.init(cfg["shape"], cfg.get("rho"), cfg.get("u"), cfg.get("flags"))
    S = oracle.run(S, cfg["tau"], steps, F=cfg.get("force"), flags=cfg.get("flags"))
    r, u = oracle.macros(S, F=cfg.get("force"), flags=cfg.get("flags"))
    return r, u, S


def fluid_mask(cfg):
    fl = cfg.get("flags")
    if fl is None:
        return np.ones(cfg["shape"], dtype=bool)
    return fl == 0


def rel_l2_u(u_gpu, u_ref, mask):
    d = (u_gpu - u_ref)[:, mask]
    r = u_ref[:, mask]
    return float(np.sqrt((d * d).sum() / (r * r).sum()))


def max_abs(a, b, mask):
    return float(np.abs(a[mask] - b[mask]).max()) if mask.any() else 0.0

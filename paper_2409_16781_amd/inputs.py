"""Seeded synthetic inputs for the lattice workloads.

This module only builds initial fields and flag masks (plain trigonometry,
seeded random numbers and geometry); it holds none of the lattice Boltzmann
arithmetic.  The same arrays feed the GPU library and the FP64 oracle.

Workloads (all lattice units):

* Taylor-Green vortex, uniform in z (the paper lists the Taylor-Green vortex
  among the mini-app's use cases, Section 3.3 "Use Cases"):
      u_x =  u0 sin(k x) cos(k y),  u_y = -u0 cos(k x) sin(k y),  u_z = 0,
      rho = 1 + (3 u0^2 / 4) (cos 2kx + cos 2ky),   k = 2 pi / n
  with x, y the integer node indices (pressure of the incompressible vortex,
  rho = 1 + 3 p for sound speed squared 1/3).
* Channel: solid planes y = 0 and y = ny - 1, periodic in x and z (no-slip
  walls, the boundary type of the paper's lid-driven cavity, Section 3.3).
* Porous channel: channel walls plus seeded random spheres to a target
  porosity.
* Batch: many porous channels of seeded random extents and relaxation times
  (``batch_domains``).
* Noise: i.i.d. uniform in [-a, a], drawn once in float64 with
  ``numpy.random.default_rng(seed)`` in C order (component, z, y, x).
"""
from __future__ import annotations

import math

import numpy as np


def tgv_fields(nx: int, ny: int, nz: int, u0: float):
    """Taylor-Green vortex (uniform in z).  Returns rho (nz,ny,nx), u (3,nz,ny,nx), float64."""
    if nx != ny:
        raise ValueError("the Taylor-Green workload uses a square x-y cross-section")
    k = 2.0 * math.pi / nx
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    sx, cx = np.sin(k * x), np.cos(k * x)
    sy, cy = np.sin(k * y), np.cos(k * y)
    ux2 = u0 * np.outer(cy, sx)            # (ny, nx): sin(kx) cos(ky)
    uy2 = -u0 * np.outer(sy, cx)           # -cos(kx) sin(ky)
    r2 = 1.0 + 0.75 * u0 * u0 * (np.cos(2 * k * x)[None, :] + np.cos(2 * k * y)[:, None])
    rho = np.broadcast_to(r2, (nz, ny, nx)).copy()
    u = np.zeros((3, nz, ny, nx))
    u[0] = ux2
    u[1] = uy2
    return rho, u


def uniform_noise(shape, amplitude: float, seed: int) -> np.ndarray:
    """i.i.d. uniform noise in [-amplitude, amplitude], float64, C order."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=shape)


def channel_flags(nx: int, ny: int, nz: int) -> np.ndarray:
    """uint8 flags (nz, ny, nx): solid planes at y = 0 and y = ny - 1."""
    f = np.zeros((nz, ny, nx), dtype=np.uint8)
    f[:, 0, :] = 1
    f[:, ny - 1, :] = 1
    return f


def random_flags(nx: int, ny: int, nz: int, fraction: float, seed: int) -> np.ndarray:
    """uint8 flags with each site solid with probability ``fraction`` (test geometry)."""
    rng = np.random.default_rng(seed)
    return (rng.random((nz, ny, nx)) < fraction).astype(np.uint8)


def sphere_flags(nx: int, ny: int, nz: int, porosity: float, seed: int,
                 rmin: float = 2.0, rmax: float = 6.0, walls: bool = True) -> np.ndarray:
    """Channel (optional walls at y = 0, ny-1) filled with random periodic spheres.

    Sphere centres are uniform over the box and radii uniform in [rmin, rmax];
    spheres are added until the fluid fraction drops to ``porosity`` or below.
    A site belongs to a sphere when its periodic (minimum-image) distance to
    the centre is at most the radius.  Each sphere is drawn only inside its
    bounding box (the sites within reach of the centre along each axis).
    """
    rng = np.random.default_rng(seed)
    f = channel_flags(nx, ny, nz) if walls else np.zeros((nz, ny, nx), dtype=np.uint8)
    total = nx * ny * nz
    solid = int(f.sum())

    def reach(c, r, n):
        # integer coordinates within distance r of c (periodic), as int64
        lo, hi = int(np.floor(c - r)), int(np.ceil(c + r))
        if hi - lo + 1 >= n:
            return np.arange(n, dtype=np.int64)
        return np.unique(np.arange(lo, hi + 1, dtype=np.int64) % n)

    for _ in range(100000):
        if 1.0 - solid / total <= porosity:
            break
        c = rng.uniform(0, 1, 3) * np.array([nx, ny, nz])
        r = rng.uniform(rmin, rmax)
        xs, ys, zs = reach(c[0], r, nx), reach(c[1], r, ny), reach(c[2], r, nz)
        dx = np.abs(xs - c[0]); dx = np.minimum(dx, nx - dx)
        dy = np.abs(ys - c[1]); dy = np.minimum(dy, ny - dy)
        dz = np.abs(zs - c[2]); dz = np.minimum(dz, nz - dz)
        inside = (dx[None, None, :] * dx[None, None, :] + dy[None, :, None] * dy[None, :, None]
                  + dz[:, None, None] * dz[:, None, None]) <= r * r
        box = np.ix_(zs, ys, xs)
        sub = f[box]
        solid += int(np.count_nonzero(inside & (sub == 0)))
        sub[inside] = 1
        f[box] = sub
    return f


def smooth_fields(xp, iz, iy, ix, n, amp: float = 0.02):
    """Analytic smooth initial fields at integer site indices (any lattice size).

    xp is numpy or torch; iz, iy, ix broadcastable index arrays (float64).
    rho = 1 + amp/4 cos(phi_3), u_x = amp sin(phi_1), u_y = amp cos(phi_2),
    u_z = amp sin(phi_3) with phases phi_k = 2 pi (a_k x + b_k y + c_k z) / n.
    Evaluated identically on the host (numpy) and on the device (torch), so
    a window of it can be rebuilt for the oracle without the whole field.
    """
    two_pi = 2.0 * math.pi / n
    p1 = two_pi * (ix + 2 * iy + 3 * iz)
    p2 = two_pi * (3 * ix + iy + 2 * iz)
    p3 = two_pi * (2 * ix + 3 * iy + iz)
    rho = 1.0 + 0.25 * amp * xp.cos(p3)
    u = xp.stack([amp * xp.sin(p1), amp * xp.cos(p2), amp * xp.sin(p3)])
    return rho, u


# --- the named workloads -------------------------------------------------------

def tgv_box(n: int = 32, u0: float = 0.01, tau: float = 0.8, steps: int = 200):
    """Periodic n^3 Taylor-Green vortex, no noise (32^3, tau 0.8, 200 steps)."""
    rho, u = tgv_fields(n, n, n, u0)
    return dict(name=f"tgv{n}", shape=(n, n, n), rho=rho, u=u, flags=None, tau=tau,
                force=(0.0, 0.0, 0.0), steps=steps)


def channel(nx: int = 256, ny: int = 128, nz: int = 128, tau: float = 0.6, g: float = 1e-6,
            steps: int = 5000, noise: float = 1e-4, seed: int = 1):
    """Force-driven channel: walls at y = 0 and ny-1, rho = 1 + U(+-noise), u = 0."""
    rho = 1.0 + uniform_noise((nz, ny, nx), noise, seed)
    u = np.zeros((3, nz, ny, nx))
    return dict(name=f"channel{nx}x{ny}x{nz}", shape=(nz, ny, nx), rho=rho, u=u,
                flags=channel_flags(nx, ny, nz), tau=tau, force=(g, 0.0, 0.0), steps=steps)


def batch_domains(count: int = 64, nmin: int = 16, nmax: int = 96, porosity: float = 0.8,
                  tau_lo: float = 0.55, tau_hi: float = 1.0, g: float = 1e-6, noise: float = 1e-4, seed: int = 3):
    """Batch of independent porous channel domains.

    Extents nx, ny, nz drawn independently and uniformly from {nmin..nmax};
    tau uniform in [tau_lo, tau_hi]; walls at y = 0 and ny-1 plus random
    spheres of radius U[2, 6] to the given porosity (sphere seed
    1000 * seed + d for domain d); force (g, 0, 0); rho = 1 + U(+-noise)
    (seed 2000 * seed + d), u = 0.  Returns a list of per-domain dicts.
    """
    rng = np.random.default_rng(seed)
    dims = rng.integers(nmin, nmax + 1, size=(count, 3))
    taus = rng.uniform(tau_lo, tau_hi, size=count)
    out = []
    for d in range(count):
        nx, ny, nz = (int(v) for v in dims[d])
        flags = sphere_flags(nx, ny, nz, porosity, 1000 * seed + d, rmin=2.0, rmax=6.0, walls=True)
        rho = 1.0 + uniform_noise((nz, ny, nx), noise, 2000 * seed + d)
        out.append(dict(name=f"batch{d}", shape=(nz, ny, nx), rho=rho, u=np.zeros((3, nz, ny, nx)),
                        flags=flags, tau=float(taus[d]), force=(g, 0.0, 0.0)))
    return out


def porous_channel(n: int = 128, porosity: float = 0.85, tau: float = 0.6, g: float = 1e-6, seed: int = 4,
                   steps: int = 500, every: int = 50):
    """n^3 porous channel for the force gradient: walls at y = 0 and n-1 plus
    random spheres (radius U[2, 6], seed) to the given porosity, uniform force
    (g, 0, 0), at rest initially (rho = 1, u = 0)."""
    flags = sphere_flags(n, n, n, porosity, seed, rmin=2.0, rmax=6.0, walls=True)
    return dict(name=f"porous{n}", shape=(n, n, n), rho=np.ones((n, n, n)), u=np.zeros((3, n, n, n)),
                flags=flags, tau=tau, force=(g, 0.0, 0.0), steps=steps, every=every)


def cavity_flags(nx: int, ny: int) -> np.ndarray:
    """uint8 flags (ny, nx) of a lid-driven cavity: walls (1) at x = 0,
    x = nx - 1 and y = 0; the lid (2) on the top row y = ny - 1 between the
    corners, which are walls."""
    f = np.zeros((ny, nx), dtype=np.uint8)
    f[0, :] = 1
    f[:, 0] = 1
    f[:, nx - 1] = 1
    f[ny - 1, 1:nx - 1] = 2
    return f


def lid_cavity(n: int = 4096, u0: float = 0.1, re: float = 1e4):
    """The paper's lid-driven cavity (Section 3.3; n x n sites, Re = 1e4):
    lid speed u0 along +x, viscosity from Re = u0 L / nu with L = n - 2 (the
    fluid width between the halfway walls), tau = 3 nu + 1/2, at rest
    initially."""
    nu = u0 * (n - 2) / re
    return dict(name=f"cavity{n}", shape=(n, n), flags=cavity_flags(n, n), tau=3.0 * nu + 0.5, lid=(u0, 0.0),
                rho=None, u=None)


def tgv_noise_box(n: int = 512, u0: float = 0.01, tau: float = 0.55, steps: int = 1000,
                  noise: float = 1e-3, seed: int = 2):
    """Periodic n^3 Taylor-Green vortex plus i.i.d. U(+-noise) on every velocity component."""
    rho, u = tgv_fields(n, n, n, u0)
    if noise:
        u += uniform_noise(u.shape, noise, seed)
    return dict(name=f"tgv{n}_noise", shape=(n, n, n), rho=rho, u=u, flags=None, tau=tau,
                force=(0.0, 0.0, 0.0), steps=steps)

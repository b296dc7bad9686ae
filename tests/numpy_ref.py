"""A second, independent FP64 implementation of one D3Q19 BGK step (tests only).

Written in a different style from the C oracle (whole-array numpy, streaming
by ``np.roll``) so that the two can pin each other on tiny lattices.  Same
method: paper Eq. 1-3 (Section 2) in the fused pull form of Section 3.1, Guo
forcing, halfway bounce-back at solid sites, periodic faces.

State layout: float64 (19, nz, ny, nx), unshifted populations.
"""
from __future__ import annotations

import itertools

import numpy as np


def _velocity_set():
    """D3Q19 in the library ordering: rest; +-x, +-y, +-z; xy, xz, yz diagonals."""
    vel = [(0, 0, 0)]
    for a in range(3):                       # axis directions, + then -
        for s in (1, -1):
            v = [0, 0, 0]
            v[a] = s
            vel.append(tuple(v))
    for a, b in ((0, 1), (0, 2), (1, 2)):    # face diagonals per plane
        for sa, sb in itertools.product((1, -1), (1, -1)):
            v = [0, 0, 0]
            v[a], v[b] = sa, sb
            vel.append(tuple(v))
    c = np.array(vel, dtype=np.int64)
    speed2 = (c * c).sum(axis=1)
    w = np.select([speed2 == 0, speed2 == 1, speed2 == 2], [1 / 3, 1 / 18, 1 / 36])
    opp = np.array([int(np.flatnonzero((c == -ci).all(axis=1))[0]) for ci in c])
    return c, w, opp


C, W, OPP = _velocity_set()


def equilibrium(rho, u):
    """f^eq for fields rho (nz,ny,nx), u (3,nz,ny,nx) -> (19,nz,ny,nx)."""
    cu = np.einsum("ia,a...->i...", C.astype(np.float64), u)
    uu = (u * u).sum(axis=0)
    return W[:, None, None, None] * rho[None] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu[None])


def step(S, tau, F=(0.0, 0.0, 0.0), flags=None):
    """One step; returns (S', rho_pre, u_pre).  Solid sites copy through."""
    omega = 1.0 / tau
    F = np.asarray(F, dtype=np.float64)
    solid = np.zeros(S.shape[1:], dtype=bool) if flags is None else flags.astype(bool)
    f = np.empty_like(S)
    for i in range(19):
        # pull: f_i(x) = S_i(x - c_i); np.roll by +c moves the value at x - c to x
        shift = (int(C[i, 2]), int(C[i, 1]), int(C[i, 0]))
        pulled = np.roll(S[i], shift, axis=(0, 1, 2))
        src_solid = np.roll(solid, shift, axis=(0, 1, 2))
        f[i] = np.where(src_solid, S[OPP[i]], pulled)
    rho = f.sum(axis=0)
    mom = np.einsum("ia,i...->a...", C.astype(np.float64), f)
    u = (mom + 0.5 * F[:, None, None, None]) / rho[None]
    feq = equilibrium(rho, u)
    cu = np.einsum("ia,a...->i...", C.astype(np.float64), u)
    cF = C.astype(np.float64) @ F                                   # (19,)
    uF = np.einsum("a,a...->...", F, u)
    src = (1 - omega / 2) * W[:, None, None, None] * (
        3 * (cF[:, None, None, None] - uF[None]) + 9 * cu * cF[:, None, None, None])
    out = f - omega * (f - feq) + src
    out = np.where(solid[None], S, out)
    rho = np.where(solid, 0.0, rho)
    u = np.where(solid[None], 0.0, u)
    return out, rho, u

"""FP64 CPU oracle for the D3Q19 BGK update (ctypes wrapper around d3q19_oracle.c).

TEST INFRASTRUCTURE ONLY: the oracle is what the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code with the HIP library and
imports nothing from it.

The method it implements is the paper's Eq. 1-3 (Section 2, "Lattice Boltzmann
Method") in the fused two-array form of Section 3.1, on the D3Q19 velocity set,
with Guo forcing and halfway bounce-back; ``d3q19_oracle.c`` lists each step
and each reading of the paper.  It also holds the adjoint of one step (the
transposed collision Jacobian and the transposed streaming) and a
checkpointed gradient of the outlet mass flux with respect to a per-site
x-force.

Array conventions (all numpy, C-contiguous):
  state S   float64, shape (19, nz, ny, nx), unshifted populations
  flags     uint8,   shape (nz, ny, nx), 0 fluid / 1 solid (None: all fluid)
  rho       float64, shape (nz, ny, nx)
  u         float64, shape (3, nz, ny, nx)  (u_x, u_y, u_z)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "d3q19_oracle.c")
_SRC2 = os.path.join(_HERE, "d2q9_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_d3q19.so")

Q = 19


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB, _SRC, _SRC2, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        i32 = ctypes.POINTER(ctypes.c_int)
        ci = ctypes.c_int
        lib.oracle_q.restype = ci
        lib.oracle_lattice.argtypes = [i32, d, i32]
        lib.oracle_feq.argtypes = [ctypes.c_double, d, d]
        lib.oracle_source.argtypes = [ctypes.c_double, d, d, d]
        lib.oracle_init.argtypes = [ci, ci, ci, u8, d, d, d]
        lib.oracle_step.argtypes = [ci, ci, ci, u8, ctypes.c_double, d, d, d, d, d, d]
        lib.oracle_run.argtypes = [ci, ci, ci, u8, ctypes.c_double, d, d, d, ci]
        lib.oracle_run.restype = ci
        lib.oracle_macros.argtypes = [ci, ci, ci, u8, d, d, d, d, d]
        lib.oracle_sums.argtypes = [ci, ci, ci, u8, d, d]
        lib.oracle2_lattice.argtypes = [i32, d, i32]
        lib.oracle2_feq.argtypes = [ctypes.c_double, d, d]
        lib.oracle2_init.argtypes = [ci, ci, u8, d, d, d]
        lib.oracle2_step.argtypes = [ci, ci, u8, ctypes.c_double, d, d, d]
        lib.oracle2_run.argtypes = [ci, ci, u8, ctypes.c_double, d, d, ci]
        lib.oracle2_run.restype = ci
        lib.oracle2_macros.argtypes = [ci, ci, u8, d, d, d]
        lib.oracle2_sums.argtypes = [ci, ci, u8, d, d]
        lib.oracle_collision_jacobian.argtypes = [ctypes.c_double, d, d, d, d]
        lib.oracle_adjoint_step.argtypes = [ci, ci, ci, u8, ctypes.c_double, d, d, d, d, d, d]
        lib.oracle_adjoint_step.restype = ci
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(flags, shape):
    if flags is None:
        return None
    assert flags.dtype == np.uint8 and flags.flags.c_contiguous and flags.shape == shape
    return flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _vec3(F):
    if F is None:
        return None
    return np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(3))


def lattice():
    """Return (c[19,3] int, w[19] float64, opp[19] int) as the oracle defines them."""
    lib = _load()
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    opp = np.zeros(Q, dtype=np.int32)
    lib.oracle_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w),
                       opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c, w, opp


def feq(rho: float, u) -> np.ndarray:
    """Eq. 2-3 equilibrium for one site."""
    out = np.zeros(Q)
    _load().oracle_feq(float(rho), _dp(_vec3(u)), _dp(out))
    return out


def source(omega: float, u, F) -> np.ndarray:
    """Guo source term S_i for one site."""
    out = np.zeros(Q)
    _load().oracle_source(float(omega), _dp(_vec3(u)), _dp(_vec3(F)), _dp(out))
    return out


def init(shape, rho=None, u=None, flags=None) -> np.ndarray:
    """S_0 = f^eq(rho, u) at fluid sites, f = w at solid sites."""
    nz, ny, nx = shape
    S = np.zeros((Q, nz, ny, nx))
    rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    _load().oracle_init(nx, ny, nz, _fp(flags, (nz, ny, nx)), _dp(rho), _dp(u), _dp(S))
    return S


def step(S, tau, F=None, flags=None, Fx_field=None, moments=False):
    """One fused step; returns S' (and (rho, u) pre-collision moments if asked)."""
    _, nz, ny, nx = S.shape
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.empty_like(S)
    rho = np.empty((nz, ny, nx)) if moments else None
    u = np.empty((3, nz, ny, nx)) if moments else None
    fx = None if Fx_field is None else np.ascontiguousarray(Fx_field, dtype=np.float64)
    _load().oracle_step(nx, ny, nz, _fp(flags, (nz, ny, nx)), 1.0 / tau, _dp(_vec3(F)), _dp(fx),
                        _dp(S), _dp(out), _dp(rho), _dp(u))
    return (out, rho, u) if moments else out


def run(S, tau, nsteps, F=None, flags=None, Fx_field=None, copy=True) -> np.ndarray:
    """n steps; returns the new state.  The input array is not modified unless
    copy=False, which advances a C-contiguous float64 S in place (one state
    less in memory for the largest lattices)."""
    _, nz, ny, nx = S.shape
    if copy:
        S = np.array(S, dtype=np.float64, order="C", copy=True)
    elif S.dtype != np.float64 or not S.flags.c_contiguous:
        raise ValueError("run(copy=False) needs a C-contiguous float64 state")
    fx = None if Fx_field is None else np.ascontiguousarray(Fx_field, dtype=np.float64)
    rc = _load().oracle_run(nx, ny, nz, _fp(flags, (nz, ny, nx)), 1.0 / tau, _dp(_vec3(F)),
                            _dp(fx), _dp(S), int(nsteps))
    if rc != 0:
        raise MemoryError("oracle_run: allocation failed")
    return S


def macros(S, F=None, flags=None, Fx_field=None):
    """(rho, u) of a stored post-collision state (Guo identity form)."""
    _, nz, ny, nx = S.shape
    S = np.ascontiguousarray(S, dtype=np.float64)
    rho = np.empty((nz, ny, nx))
    u = np.empty((3, nz, ny, nx))
    fx = None if Fx_field is None else np.ascontiguousarray(Fx_field, dtype=np.float64)
    _load().oracle_macros(nx, ny, nz, _fp(flags, (nz, ny, nx)), _dp(_vec3(F)), _dp(fx), _dp(S),
                          _dp(rho), _dp(u))
    return rho, u


def sums(S, flags=None) -> np.ndarray:
    """[sum S, sum c_x S, sum c_y S, sum c_z S] over fluid sites."""
    _, nz, ny, nx = S.shape
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.zeros(4)
    _load().oracle_sums(nx, ny, nz, _fp(flags, (nz, ny, nx)), _dp(S), _dp(out))
    return out


def collision_jacobian(f, tau, F):
    """(J[19, 19], dFx[19]): J[i, j] = dC_i/df_j and dC_i/dF_x of one site's
    collision for pre-collision populations f and force density F."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(Q)
    J = np.zeros((Q, Q))
    dF = np.zeros(Q)
    omega = 0.0 if np.isinf(tau) else 1.0 / tau
    _load().oracle_collision_jacobian(omega, _dp(f), _dp(_vec3(F)), _dp(J), _dp(dF))
    return J, dF


def adjoint_step(S_n, lam_next, tau, F=None, flags=None, Fx_field=None):
    """Adjoint of the step taken from S_n: returns (dJ/dS_n, dJ/dF_x increment)
    given lam_next = dJ/dS_{n+1}."""
    _, nz, ny, nx = S_n.shape
    S_n = np.ascontiguousarray(S_n, dtype=np.float64)
    lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
    out = np.empty_like(S_n)
    g = np.zeros((nz, ny, nx))
    fx = None if Fx_field is None else np.ascontiguousarray(Fx_field, dtype=np.float64)
    omega = 0.0 if np.isinf(tau) else 1.0 / tau
    rc = _load().oracle_adjoint_step(nx, ny, nz, _fp(flags, (nz, ny, nx)), omega, _dp(_vec3(F)), _dp(fx),
                                     _dp(S_n), _dp(lam_next), _dp(out), _dp(g))
    if rc != 0:
        raise MemoryError("oracle_adjoint_step: allocation failed")
    return out, g


def outlet_flux(S, F=None, flags=None, Fx_field=None):
    """J = sum over the fluid sites of the plane x = nx - 1 of rho u_x
    (= sum_i c_ix S_i - F_x / 2 there), for a stored state S."""
    rho, u = macros(S, F=F, flags=flags, Fx_field=Fx_field)
    return float((rho[:, :, -1] * u[0, :, :, -1]).sum())


def grad_outlet_flux(S0, tau, nsteps, F=None, flags=None, Fx_field=None, every=None):
    """J(S_nsteps) = outlet_flux after nsteps steps from S0, and dJ/dF_x for
    every site (the per-site x-force is F[0] + Fx_field).  The forward states
    are kept at every ``every`` steps (all of them when None) and each
    segment is recomputed from its checkpoint for the backward sweep."""
    _, nz, ny, nx = S0.shape
    every = nsteps if every is None else int(every)
    fx = np.zeros((nz, ny, nx)) if Fx_field is None else np.ascontiguousarray(Fx_field, dtype=np.float64)
    C = lattice()[0]
    fluid = np.ones((nz, ny, nx), bool) if flags is None else flags == 0
    checkpoints = {}
    S = np.array(S0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        if n % every == 0:
            checkpoints[n] = S.copy()
        S = step(S, tau, F=F, flags=flags, Fx_field=fx)
    J = outlet_flux(S, F=F, flags=flags, Fx_field=fx)
    # seed: dJ/dS_N = c_ix at the outlet's fluid sites; direct term -1/2 per outlet site
    lam = np.zeros_like(S)
    out_mask = np.zeros((nz, ny, nx), bool)
    out_mask[:, :, -1] = fluid[:, :, -1]
    for i in range(Q):
        lam[i][out_mask] = C[i, 0]
    grad = np.zeros((nz, ny, nx))
    grad[out_mask] -= 0.5
    for start in sorted(checkpoints, reverse=True):
        stop = min(start + every, nsteps)
        states = [checkpoints[start]]
        for n in range(start, stop - 1):
            states.append(step(states[-1], tau, F=F, flags=flags, Fx_field=fx))
        for n in range(stop - 1, start - 1, -1):
            lam, g = adjoint_step(states[n - start], lam, tau, F=F, flags=flags, Fx_field=fx)
            grad += g
    return J, grad


# --------------------------------------------------------------- D2Q9 -------
# The two-dimensional D2Q9 oracle (d2q9_oracle.c): state (9, ny, nx), flags
# (ny, nx) with 0 fluid, 1 wall, 2 lid moving with velocity `lid`.

Q2 = 9


def d2_lattice():
    c = np.zeros((Q2, 2), dtype=np.int32)
    w = np.zeros(Q2)
    opp = np.zeros(Q2, dtype=np.int32)
    _load().oracle2_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w),
                            opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c, w, opp


def d2_feq(rho, u):
    out = np.zeros(Q2)
    _load().oracle2_feq(float(rho), _dp(np.ascontiguousarray(np.asarray(u, np.float64).reshape(2))), _dp(out))
    return out


def d2_init(shape, rho=None, u=None, flags=None):
    ny, nx = shape
    S = np.zeros((Q2, ny, nx))
    rho = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    _load().oracle2_init(nx, ny, _fp(flags, (ny, nx)), _dp(rho), _dp(u), _dp(S))
    return S


def _lid(lid):
    return np.ascontiguousarray(np.asarray((0.0, 0.0) if lid is None else lid, np.float64).reshape(2))


def d2_step(S, tau, flags=None, lid=None):
    _, ny, nx = S.shape
    S = np.ascontiguousarray(S, dtype=np.float64)
    out = np.empty_like(S)
    omega = 0.0 if np.isinf(tau) else 1.0 / tau
    _load().oracle2_step(nx, ny, _fp(flags, (ny, nx)), omega, _dp(_lid(lid)), _dp(S), _dp(out))
    return out


def d2_run(S, tau, nsteps, flags=None, lid=None):
    _, ny, nx = S.shape
    S = np.array(S, dtype=np.float64, order="C", copy=True)
    omega = 0.0 if np.isinf(tau) else 1.0 / tau
    if _load().oracle2_run(nx, ny, _fp(flags, (ny, nx)), omega, _dp(_lid(lid)), _dp(S), int(nsteps)) != 0:
        raise MemoryError("oracle2_run: allocation failed")
    return S


def d2_macros(S, flags=None):
    _, ny, nx = S.shape
    S = np.ascontiguousarray(S, dtype=np.float64)
    rho = np.empty((ny, nx))
    u = np.empty((2, ny, nx))
    _load().oracle2_macros(nx, ny, _fp(flags, (ny, nx)), _dp(S), _dp(rho), _dp(u))
    return rho, u


def d2_sums(S, flags=None):
    _, ny, nx = S.shape
    out = np.zeros(3)
    _load().oracle2_sums(nx, ny, _fp(flags, (ny, nx)), _dp(np.ascontiguousarray(S, np.float64)), _dp(out))
    return out


def run_window(rho, u, flags, tau, nsteps, centres, F=None, shape=None, fields=None):
    """Light-cone evaluation of single sites after ``nsteps`` steps.

    A site's value after n steps depends only on the initial state within
    L-infinity distance n (every D3Q19 velocity moves at most one site per
    axis per step).  For each centre (z, y, x) this cuts the (2n+1)-wide
    window around it out of the periodic initial fields (the whole axis when
    it is no wider than that), runs the oracle on the window alone and returns
    (rho, u) at the centre.  Errors from the window's own artificial wrap
    travel inward one site per step and reach distance n-1 from the edge at
    most, so the centre is exact.  The initial fields come either from full
    arrays (rho, u, flags) or, with ``fields`` and ``shape`` = (nz, ny, nx),
    from a function fields(iz, iy, ix) -> (rho, u) evaluated on the window's
    periodic site indices (then flags is None).  Returns rho[k], u[k, 3].
    """
    nz, ny, nx = shape if shape is not None else rho.shape
    W = 2 * nsteps + 1
    out_r = np.empty(len(centres))
    out_u = np.empty((len(centres), 3))
    for k, (cz, cy, cx) in enumerate(centres):
        idx = []
        cen = []
        for c, n in ((cz, nz), (cy, ny), (cx, nx)):
            if n <= W:
                idx.append(np.arange(n))
                cen.append(c)
            else:
                idx.append((np.arange(W) + c - nsteps) % n)
                cen.append(nsteps)
        iz, iy, ix = np.ix_(*idx)
        if fields is not None:
            r_w, u_w = fields(iz.astype(np.float64), iy.astype(np.float64), ix.astype(np.float64))
            r_w = np.ascontiguousarray(np.broadcast_to(r_w, (len(idx[0]), len(idx[1]), len(idx[2]))))
            u_w = np.ascontiguousarray(np.broadcast_to(u_w, (3, len(idx[0]), len(idx[1]), len(idx[2]))))
            f_w = None
        else:
            r_w = np.ascontiguousarray(rho[iz, iy, ix], dtype=np.float64)
            u_w = np.ascontiguousarray(u[:, iz, iy, ix], dtype=np.float64)
            f_w = None if flags is None else np.ascontiguousarray(flags[iz, iy, ix])
        S = init(r_w.shape, r_w, u_w, f_w)
        S = run(S, tau, nsteps, F=F, flags=f_w)
        r_o, u_o = macros(S, F=F, flags=f_w)
        out_r[k] = r_o[cen[0], cen[1], cen[2]]
        out_u[k] = u_o[:, cen[0], cen[1], cen[2]]
    return out_r, out_u

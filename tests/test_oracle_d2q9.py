"""Pins of the two-dimensional D2Q9 oracle (the paper's lid-driven cavity
workload), CPU only.  Each compares the oracle with something computed
without it: lattice identities, a closed form on one site, a pure-Python
permutation, the exact plane Couette profile between a fixed wall and the
moving lid, exact mass conservation of the cavity, and an independent numpy
implementation."""
import math

import numpy as np
import pytest

import oracle
from paper_2409_16781_amd import inputs


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


def test_d2q9_lattice_isotropy_and_opposites():
    c, w, opp = oracle.d2_lattice()
    cf = c.astype(np.float64)
    assert abs(w.sum() - 1.0) < 1e-16
    assert np.allclose(w @ cf, 0.0, atol=1e-17)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, cf, cf), np.eye(2) / 3.0, atol=1e-16)
    four = np.einsum("i,ia,ib,ic,id->abcd", w, cf, cf, cf, cf)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(four, iso, atol=1e-16)
    for i in range(9):
        assert np.array_equal(c[opp[i]], -c[i])


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0)), (1.03, (0.05, -0.02)), (0.97, (-0.1, 0.07))])
def test_d2q9_equilibrium_moments(rho, u):
    c, w, _ = oracle.d2_lattice()
    cf = c.astype(np.float64)
    f = oracle.d2_feq(rho, u)
    u = np.array(u)
    assert abs(f.sum() - rho) < 1e-15
    assert np.allclose(cf.T @ f, rho * u, atol=1e-16)
    assert np.allclose(np.einsum("ia,ib,i->ab", cf, cf, f), rho / 3.0 * np.eye(2) + rho * np.outer(u, u), atol=1e-16)


def test_single_site_relaxes_by_the_closed_form():
    """A 1x1 periodic lattice streams onto itself: S_n = feq + (1 - omega)^n (S_0 - feq)."""
    rng = np.random.default_rng(1)
    S0 = (oracle.d2_feq(1.02, (0.03, -0.01)) + rng.uniform(-1e-3, 1e-3, 9)).reshape(9, 1, 1)
    c, _, _ = oracle.d2_lattice()
    rho = S0.sum()
    u = (c.T.astype(np.float64) @ S0.reshape(9)) / rho
    feq = oracle.d2_feq(rho, u)
    tau = 0.8
    S = oracle.d2_run(S0, tau, 7)
    assert np.allclose(S.reshape(9), feq + (1 - 1 / tau) ** 7 * (S0.reshape(9) - feq), atol=1e-15)


def _python_stream(S, flags):
    """omega = 0, lid at rest: pull streaming with halfway bounce-back, element by element."""
    c, _, opp = oracle.d2_lattice()
    _, ny, nx = S.shape
    out = S.copy()
    for y in range(ny):
        for x in range(nx):
            if flags[y, x]:
                continue
            for i in range(9):
                xs, ys = (x - c[i, 0]) % nx, (y - c[i, 1]) % ny
                out[i, y, x] = S[opp[i], y, x] if flags[ys, xs] else S[i, ys, xs]
    return out


def test_pure_streaming_is_a_permutation():
    flags = inputs.cavity_flags(9, 7)
    rng = np.random.default_rng(2)
    S = rng.uniform(0.0, 0.2, (9, 7, 9))
    ref = S
    for _ in range(3):
        ref = _python_stream(ref, flags)
    out = oracle.d2_run(S, math.inf, 3, flags=flags, lid=(0.0, 0.0))
    m = flags == 0
    assert np.array_equal(out[:, m], ref[:, m])


@pytest.mark.parametrize("tau", [0.6, 1.0])
def test_plane_couette_profile_is_exact(tau):
    """Fixed wall at y = 0, lid at y = ny - 1 moving with U, periodic in x: the
    steady profile is linear between the halfway walls, u_x(y) = U (y - 1/2) / H
    with H = ny - 2, and BGK with halfway bounce-back reproduces it exactly."""
    ny, U = 18, 0.05
    flags = np.zeros((ny, 1), np.uint8)
    flags[0] = 1
    flags[-1] = 2
    S = oracle.d2_run(oracle.d2_init((ny, 1), flags=flags), tau, 30000, flags=flags, lid=(U, 0.0))
    rho, u = oracle.d2_macros(S, flags=flags)
    y = np.arange(1, ny - 1)
    assert np.abs(u[0, 1:-1, 0] - U * (y - 0.5) / (ny - 2)).max() < 1e-11
    assert np.abs(u[1, 1:-1, 0]).max() < 1e-12


def test_cavity_conserves_mass():
    """The lid's momentum terms cancel over the lid (the two corner sites
    cancel each other), so the total mass stays exact to rounding."""
    flags = inputs.cavity_flags(32, 32)
    S0 = oracle.d2_init((32, 32), flags=flags)
    S = oracle.d2_run(S0, 0.6, 300, flags=flags, lid=(0.1, 0.0))
    m0, m1 = oracle.d2_sums(S0, flags)[0], oracle.d2_sums(S, flags)[0]
    assert abs(m1 - m0) <= 1e-13 * m0
    rho, u = oracle.d2_macros(S, flags=flags)
    assert u[0, -2, 16] > 0.0  # the fluid under the lid is dragged along +x


def _numpy_step(S, tau, flags, lid):
    """Independent numpy D2Q9 step: np.roll streaming, bounce-back and the lid term by masks."""
    c = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, 1], [1, -1], [-1, 1], [-1, -1]])
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    opp = [0, 2, 1, 4, 3, 8, 7, 6, 5]
    f = np.empty_like(S)
    for i in range(9):
        pulled = np.roll(S[i], shift=(c[i, 1], c[i, 0]), axis=(0, 1))
        src_flag = np.roll(flags, shift=(c[i, 1], c[i, 0]), axis=(0, 1))
        bounce = S[opp[i]] + np.where(src_flag == 2, 6 * w[i] * (c[i] @ np.array(lid)), 0.0)
        f[i] = np.where(src_flag > 0, bounce, pulled)
    rho = f.sum(0)
    u = np.einsum("ia,iyx->ayx", c.astype(float), f) / rho
    cu = np.einsum("ia,ayx->iyx", c.astype(float), u)
    feq = w[:, None, None] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u ** 2).sum(0))
    out = f - (f - feq) / tau
    return np.where(flags[None] > 0, S, out)


def test_oracle_matches_independent_numpy_step():
    flags = inputs.cavity_flags(13, 11)
    rng = np.random.default_rng(3)
    S = oracle.d2_init((11, 13), rho=1 + rng.uniform(-1e-3, 1e-3, (11, 13)),
                       u=rng.uniform(-0.05, 0.05, (2, 11, 13)), flags=flags)
    a, b = S, S
    for _ in range(20):
        a = oracle.d2_step(a, 0.7, flags=flags, lid=(0.08, 0.0))
        b = _numpy_step(b, 0.7, flags, (0.08, 0.0))
    m = flags == 0
    assert np.abs(a[:, m] - b[:, m]).max() < 1e-14


# ------------------------------------------------------- oracle2_sums pins --
# The velocity order of reading 20 written out here, not taken from the oracle.
D2Q9_C = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]


def test_sums_of_single_populations_follow_the_velocity_order():
    """One nonzero population i at one fluid site: the totals are
    (v, c_ix v, c_iy v) with c_i from the written-out order, and a solid site's
    values are left out."""
    flags = np.zeros((3, 4), np.uint8)
    flags[2, 3] = 1
    for i, (cx, cy) in enumerate(D2Q9_C):
        S = np.zeros((9, 3, 4))
        S[i, 1, 2] = 0.375
        S[i, 2, 3] = 5.0  # solid site: excluded
        assert np.array_equal(oracle.d2_sums(S, flags), [0.375, cx * 0.375, cy * 0.375])


def test_sums_of_a_uniform_flow_are_mass_times_velocity():
    """A periodic box at uniform (rho, u): the equilibrium carries exactly rho u
    per site (second-order Maxwell-Boltzmann truncation), so the totals are
    N (rho, rho u_x, rho u_y); u_x and u_y differ in size and sign, so a
    swapped or mis-signed component fails."""
    ny, nx, rho, u = 5, 7, 1.01, (0.03, -0.02)
    S = oracle.d2_init((ny, nx), rho=np.full((ny, nx), rho),
                       u=np.stack([np.full((ny, nx), u[0]), np.full((ny, nx), u[1])]))
    n = nx * ny
    assert np.allclose(oracle.d2_sums(S), [n * rho, n * rho * u[0], n * rho * u[1]], rtol=0, atol=1e-13)
    # invariant under steps (uniform flow on a periodic box is a fixed point)
    S = oracle.d2_run(S, 0.7, 25)
    assert np.allclose(oracle.d2_sums(S), [n * rho, n * rho * u[0], n * rho * u[1]], rtol=0, atol=1e-12)


def test_sums_of_the_couette_strip_equal_the_exact_profile_integral():
    """Steady plane Couette flow between the wall at y = 0 and the lid at
    y = ny - 1 (speed U): rho = 1 (uniform pressure, mass exact up to FP64 rounding), and
    u_x(y) = U (y - 1/2) / H on the H = ny - 2 fluid rows, so the total
    x-momentum is U/H * sum_{y=1..H} (y - 1/2) = U H / 2 per column, and the
    y-momentum is zero."""
    ny, nx, U = 18, 3, 0.05
    flags = np.zeros((ny, nx), np.uint8)
    flags[0] = 1
    flags[-1] = 2
    S = oracle.d2_run(oracle.d2_init((ny, nx), flags=flags), 0.8, 20000, flags=flags, lid=(U, 0.0))
    H = ny - 2
    mass, px, py = oracle.d2_sums(S, flags)
    assert abs(mass - nx * H) < 1e-9  # FP64 rounding over 20000 steps: ~5e-11
    assert abs(px - nx * U * H / 2) < 1e-10
    assert abs(py) < 1e-12

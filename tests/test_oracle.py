"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test names the property it checks and the passage of the paper it
follows: Eq. 1-3 (Section 2, "Lattice Boltzmann Method"), the fused two-array
scheme (Section 3.1, "Computational Description") and the use cases
(Section 3.3: Taylor-Green vortex, no-slip walls).  None of these checks
re-types the oracle's formulas: they use closed-form solutions, conservation
laws, exact permutations, symmetry, and an independent implementation.
"""
import math

import numpy as np
import pytest

import oracle
import numpy_ref
from paper_2409_16781_amd import inputs


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ---------------------------------------------------------------- lattice ----

def test_velocity_set_is_d3q19_and_isotropic():
    """D3Q19: weights fixed by the isotropy conditions up to 4th order."""
    c, w, opp = oracle.lattice()
    c = c.astype(np.float64)
    speed2 = (c * c).sum(1)
    assert sorted(speed2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in c.astype(int)}) == 19
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(w @ c).max() < 1e-15
    I = np.eye(3)
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.abs(m2 - I / 3).max() < 1e-15
    m3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(m3).max() < 1e-15
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
           + np.einsum("ad,bc->abcd", I, I)) / 9
    assert np.abs(m4 - iso).max() < 1e-15
    for i in range(19):
        assert (c[opp[i]] == -c[i]).all()
        assert w[opp[i]] == w[i]


def test_velocity_order_matches_library_order():
    """The population order is part of the library's raw-state interface."""
    c, _, _ = oracle.lattice()
    assert (c == numpy_ref.C).all()
    # halo sets for a z-slab split: c_z = +1 and c_z = -1
    assert np.flatnonzero(c[:, 2] == 1).tolist() == [5, 11, 13, 15, 17]
    assert np.flatnonzero(c[:, 2] == -1).tolist() == [6, 12, 14, 16, 18]


# ------------------------------------------------------------ Eq. 2-3 pins ----

def test_equilibrium_moments():
    """Eq. 2-3 read with c_s^2 = 1/3: the first three moments of f^eq are
    rho, rho u and rho/3 I + rho u u (what the second-order Maxwell-Boltzmann
    truncation must give); the third moment is (rho/3)(u d + d u + ...)."""
    c, _, _ = oracle.lattice()
    c = c.astype(np.float64)
    rng = np.random.default_rng(11)
    for _ in range(20):
        rho = 1 + 0.2 * rng.standard_normal()
        u = 0.1 * rng.standard_normal(3)
        f = oracle.feq(rho, u)
        assert abs(f.sum() - rho) < 1e-15
        assert np.abs(c.T @ f - rho * u).max() < 1e-16
        m2 = np.einsum("i,ia,ib->ab", f, c, c)
        assert np.abs(m2 - (rho / 3 * np.eye(3) + rho * np.outer(u, u))).max() < 1e-15
        m3 = np.einsum("i,ia,ib,ic->abc", f, c, c, c)
        I = np.eye(3)
        exp3 = rho / 3 * (np.einsum("ab,c->abc", I, u) + np.einsum("ac,b->abc", I, u)
                          + np.einsum("bc,a->abc", I, u))
        assert np.abs(m3 - exp3).max() < 1e-15


def test_guo_source_moments():
    """Source term of Eq. 1 (Guo reading): zeroth moment 0, first moment
    (1 - omega/2) F, second moment (1 - omega/2)(u F + F u)."""
    c, _, _ = oracle.lattice()
    c = c.astype(np.float64)
    rng = np.random.default_rng(12)
    for _ in range(20):
        omega = rng.uniform(0.5, 1.9)
        u = 0.1 * rng.standard_normal(3)
        F = 1e-3 * rng.standard_normal(3)
        s = oracle.source(omega, u, F)
        k = 1 - omega / 2
        assert abs(s.sum()) < 1e-18
        assert np.abs(c.T @ s - k * F).max() < 1e-18
        m2 = np.einsum("i,ia,ib->ab", s, c, c)
        assert np.abs(m2 - k * (np.outer(u, F) + np.outer(F, u))).max() < 1e-18


def test_collision_budget_single_site():
    """On a 1x1x1 periodic lattice streaming is the identity, so one step is
    one collision: mass is kept and momentum gains exactly F."""
    c, _, _ = oracle.lattice()
    c = c.astype(np.float64)
    rng = np.random.default_rng(13)
    for tau in (0.55, 0.8, 1.7):
        S = (oracle.init((1, 1, 1), np.array([[[1.02]]]), np.array([0.03, -0.02, 0.01]).reshape(3, 1, 1, 1))
             + 1e-3 * rng.standard_normal((19, 1, 1, 1)))
        F = np.array([1e-4, -2e-4, 3e-5])
        out = oracle.step(S, tau, F=F)
        assert abs(out.sum() - S.sum()) < 1e-15
        assert np.abs(c.T @ out[:, 0, 0, 0] - (c.T @ S[:, 0, 0, 0] + F)).max() < 1e-16


def test_single_site_relaxation_closed_form():
    """1x1x1 lattice, F = 0: rho and u stay fixed, so
    S_n = f^eq + (1 - omega)^n (S_0 - f^eq) exactly."""
    rng = np.random.default_rng(14)
    S0 = oracle.feq(1.0, [0.05, 0.0, -0.03]).reshape(19, 1, 1, 1) * (1 + 0.05 * rng.random((19, 1, 1, 1)))
    rho = S0.sum()
    c = numpy_ref.C.astype(np.float64)
    u = c.T @ S0[:, 0, 0, 0] / rho
    fe = numpy_ref.equilibrium(np.array([[[rho]]]), u.reshape(3, 1, 1, 1))
    for tau in (0.6, 1.0, 1.9):
        om = 1 / tau
        for n in (1, 5, 17):
            Sn = oracle.run(S0, tau, n)
            exp = fe + (1 - om) ** n * (S0 - fe)
            assert np.abs(Sn - exp).max() < 2e-15, (tau, n)


# ------------------------------------------------------- streaming (Sec 3.1) --

def _brute_force_stream(S, flags):
    """Pure-Python pull streaming with halfway bounce-back (omega = 0)."""
    _, nz, ny, nx = S.shape
    c, opp = numpy_ref.C, numpy_ref.OPP
    out = S.copy()
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if flags is not None and flags[z, y, x]:
                    continue
                for i in range(19):
                    zs, ys, xs = (z - c[i, 2]) % nz, (y - c[i, 1]) % ny, (x - c[i, 0]) % nx
                    if flags is not None and flags[zs, ys, xs]:
                        out[i, z, y, x] = S[opp[i], z, y, x]
                    else:
                        out[i, z, y, x] = S[i, zs, ys, xs]
    return out


@pytest.mark.parametrize("with_walls", [False, True])
def test_pure_streaming_is_exact_permutation(with_walls):
    """omega = 0 (tau = infinity) and F = 0: one step is a permutation of the
    stored values (shift plus reflection at solid neighbours), bit-exact."""
    rng = np.random.default_rng(15)
    shape = (4, 3, 5)
    flags = inputs.random_flags(5, 3, 4, 0.25, 16) if with_walls else None
    S = rng.random((19,) + shape)
    out = oracle.step(S, np.inf, flags=flags)
    ref = _brute_force_stream(S, flags)
    fl = np.zeros(shape, bool) if flags is None else flags.astype(bool)
    assert np.array_equal(out[:, ~fl], ref[:, ~fl])


def test_pure_streaming_returns_after_one_period():
    """On an all-fluid periodic L^3 box with omega = 0, every population
    travels one site per step and is back at its start after L steps."""
    rng = np.random.default_rng(17)
    L = 6
    S = rng.random((19, L, L, L))
    assert np.array_equal(oracle.run(S, np.inf, L), S)
    assert not np.array_equal(oracle.run(S, np.inf, L - 1), S)


def test_wall_reflection_returns_after_round_trip():
    """omega = 0 in a channel of width H (walls at y = 0 and H+1), a
    population moving in +-y (and nothing in x, z: nx = nz = 1) returns to its
    start after 2H steps (H steps out, reflection, H steps back)."""
    rng = np.random.default_rng(18)
    H = 5
    flags = inputs.channel_flags(1, H + 2, 1)
    S = rng.random((19, 1, H + 2, 1))
    out = oracle.run(S, np.inf, 2 * H, flags=flags)
    assert np.array_equal(out[:, 0, 1:-1, 0], S[:, 0, 1:-1, 0])


# ---------------------------------------------------------- conservation ----

def test_mass_conservation_with_walls_and_force():
    rng = np.random.default_rng(19)
    n = 10
    flags = inputs.random_flags(n, n, n, 0.15, 20)
    rho = 1 + 1e-3 * rng.standard_normal((n, n, n))
    u = 0.02 * rng.standard_normal((3, n, n, n))
    S = oracle.init((n, n, n), rho, u, flags)
    M0 = oracle.sums(S, flags)[0]
    S = oracle.run(S, 0.57, 150, F=(2e-5, -1e-5, 5e-6), flags=flags)
    M1 = oracle.sums(S, flags)[0]
    assert abs(M1 - M0) / M0 < 1e-13


def test_rest_state_and_uniform_flow_are_invariant():
    n = 6
    S = oracle.init((n, n, n))
    assert np.abs(oracle.run(S, 0.7, 20) - S).max() < 1e-15
    u = np.zeros((3, n, n, n))
    u[0], u[1], u[2] = 0.05, -0.02, 0.01
    S = oracle.init((n, n, n), None, u)
    assert np.abs(oracle.run(S, 0.6, 20) - S).max() < 1e-15


def test_momentum_grows_by_force_per_step_without_walls():
    rng = np.random.default_rng(21)
    n = 7
    rho = 1 + 1e-3 * rng.standard_normal((n, n, n))
    u = 0.01 * rng.standard_normal((3, n, n, n))
    S = oracle.init((n, n, n), rho, u)
    F = np.array([3e-6, -1e-6, 2e-6])
    P0 = oracle.sums(S)[1:]
    steps = 25
    P1 = oracle.sums(oracle.run(S, 0.65, steps, F=F))[1:]
    assert np.abs(P1 - (P0 + steps * n ** 3 * F)).max() < 1e-13


# ------------------------------------------------------ macros convention ----

def test_macros_of_state_equal_precollision_moments():
    """rho = sum S_n and u = (sum c S_n - F/2)/rho equal the pre-collision
    moments gathered in step n (mass kept by collision, Guo adds exactly F)."""
    rng = np.random.default_rng(22)
    shape = (5, 6, 7)
    flags = inputs.random_flags(7, 6, 5, 0.2, 23)
    S = oracle.init(shape, 1 + 1e-3 * rng.standard_normal(shape), 0.02 * rng.standard_normal((3,) + shape), flags)
    F = (1e-4, 2e-5, -3e-5)
    S1, r_pre, u_pre = oracle.step(S, 0.66, F=F, flags=flags, moments=True)
    r, u = oracle.macros(S1, F=F, flags=flags)
    assert np.abs(r - r_pre).max() < 1e-15
    assert np.abs(u - u_pre).max() < 1e-16


# -------------------------------------------------- Taylor-Green (Sec. 3.3) ---

def _tgv_amplitude(u, k):
    nx = u.shape[-1]
    x = np.arange(nx)
    mode = np.outer(np.cos(k * x), np.sin(k * x))  # (y, x): sin(kx) cos(ky)
    return (u[0] * mode[None]).sum() / (mode * mode).sum() / u.shape[1]


def _tgv_decay_fit(n, tau, steps, u0=0.01, nz=1):
    rho, u = inputs.tgv_fields(n, n, nz, u0)
    S = oracle.init((nz, n, n), rho, u)
    k = 2 * math.pi / n
    ts, amps = [], []
    t = 0
    for target in np.linspace(steps // 20, steps, 8).astype(int):
        S = oracle.run(S, tau, int(target - t))
        t = int(target)
        _, uu = oracle.macros(S)
        ts.append(t)
        amps.append(_tgv_amplitude(uu, k))
    slope = np.polyfit(ts, np.log(amps), 1)[0]
    nu_fit = -slope / (2 * k * k)
    return nu_fit, (tau - 0.5) / 3


def test_taylor_green_decay_rate_32():
    """Taylor-Green vortex on the 32^3 periodic box, tau = 0.8: the mode
    decays as exp(-2 nu k^2 t) with nu = (tau - 1/2)/3 (to 2%)."""
    nu_fit, nu = _tgv_decay_fit(32, 0.8, 200, nz=32)
    assert abs(nu_fit / nu - 1) < 0.02


def test_taylor_green_error_is_second_order():
    """Halving the grid spacing (same diffusive time) cuts the decay-rate
    error about four times: second-order accuracy."""
    e32 = abs(np.subtract(*_tgv_decay_fit(32, 0.8, 200)) / _tgv_decay_fit(32, 0.8, 200)[1])
    nu64, nu = _tgv_decay_fit(64, 0.8, 800)
    e64 = abs(nu64 / nu - 1)
    assert 3.0 < e32 / e64 < 5.0


def test_z_uniform_state_reduces_to_one_plane_bit_exact():
    """A state uniform in z evolves as the nz = 1 lattice, in every z plane,
    bit for bit (each site does the same arithmetic)."""
    rho, u = inputs.tgv_fields(16, 16, 6, 0.02)
    S3 = oracle.run(oracle.init((6, 16, 16), rho, u), 0.55, 30)
    S1 = oracle.run(oracle.init((1, 16, 16), rho[:1], u[:, :1]), 0.55, 30)
    for z in range(6):
        assert np.array_equal(S3[:, z], S1[:, 0])


# ---------------------------------------------------------- channel flows ----

def test_channel_startup_matches_series_solution():
    """Force-driven start-up between no-slip walls: u_t = nu u_yy + g with
    u = 0 at y' = 0, H has the series solution
        u = g y'(H - y')/(2 nu) - sum_{n odd} 4 g H^2/(nu pi^3 n^3) sin(n pi y'/H) exp(-n^2 pi^2 nu t/H^2).
    Channel of the 256x128x128 workload reduced to its x-z average (nx = nz = 1,
    noise-free): H = 126, tau = 0.6, g = 1e-6, 5000 steps; with the Guo
    convention the macroscopic velocity of step n sits at t = n - 1/2."""
    tau, g, ny, T = 0.6, 1e-6, 128, 5000
    H, nu = ny - 2, (tau - 0.5) / 3
    flags = inputs.channel_flags(1, ny, 1)
    S = oracle.run(oracle.init((1, ny, 1), flags=flags), tau, T, F=(g, 0, 0), flags=flags)
    _, u = oracle.macros(S, F=(g, 0, 0), flags=flags)
    ux = u[0, 0, 1:-1, 0]
    y = np.arange(1, ny - 1) - 0.5
    t = T - 0.5
    ser = g / (2 * nu) * y * (H - y)
    for n in range(1, 4001, 2):
        ser -= 4 * g * H * H / (nu * math.pi ** 3 * n ** 3) * np.sin(n * math.pi * y / H) * math.exp(
            -n * n * math.pi ** 2 * nu * t / (H * H))
    assert abs(ser[62] - 4.99881e-3) < 1e-8          # centre value of the series itself
    assert abs(ux[62] / ser[62] - 1) < 1e-5
    assert np.linalg.norm(ux - ser) / np.linalg.norm(ser) < 1e-3


@pytest.mark.parametrize("tau", [0.6, 0.8, 0.5 + math.sqrt(3) / 4, 1.0, 1.5])
def test_steady_poiseuille_curvature_and_slip(tau):
    """Steady force-driven Poiseuille flow, halfway bounce-back: the profile is
    an exact parabola of curvature -g/nu, offset by a constant slip
    u_s = g (16 (tau - 1/2)^2 - 3) / (24 nu), which vanishes at
    tau = 1/2 + sqrt(3)/4 (the known exact-wall point of BGK bounce-back)."""
    H, g = 20, 1e-6
    ny = H + 2
    nu = (tau - 0.5) / 3
    flags = inputs.channel_flags(1, ny, 1)
    S = oracle.run(oracle.init((1, ny, 1), flags=flags), tau, int(20 * H * H / nu), F=(g, 0, 0), flags=flags)
    _, u = oracle.macros(S, F=(g, 0, 0), flags=flags)
    ux = u[0, 0, 1:-1, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    assert np.abs(d2 / (-g / nu) - 1).max() < 1e-6
    y = np.arange(1, ny - 1) - 0.5
    slip = ux - g / (2 * nu) * y * (H - y)
    expect = g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    assert np.abs(slip - expect).max() < 1e-6 * g / nu * H * H / 8


def test_channel_profile_mirror_symmetry():
    ny = 24
    flags = inputs.channel_flags(3, ny, 2)
    S = oracle.run(oracle.init((2, ny, 3), flags=flags), 0.7, 300, F=(1e-5, 0, 0), flags=flags)
    _, u = oracle.macros(S, F=(1e-5, 0, 0), flags=flags)
    prof = u[0, 0, :, 0]
    assert np.abs(prof - prof[::-1]).max() < 1e-14


# ------------------------------------------------ independent implementation --

@pytest.mark.parametrize("tau", [0.55, 1.0])
def test_oracle_matches_numpy_reference(tau):
    rng = np.random.default_rng(24)
    shape = (6, 7, 5)
    flags = inputs.random_flags(5, 7, 6, 0.2, 25)
    F = (2e-4, -1e-4, 5e-5)
    S = oracle.init(shape, 1 + 1e-2 * rng.standard_normal(shape), 0.03 * rng.standard_normal((3,) + shape), flags)
    Sn = S.copy()
    for _ in range(6):
        S, r1, u1 = oracle.step(S, tau, F=F, flags=flags, moments=True)
        Sn, r2, u2 = numpy_ref.step(Sn, tau, F=F, flags=flags)
    fl = flags.astype(bool)
    assert np.abs(S[:, ~fl] - Sn[:, ~fl]).max() < 1e-14 * np.abs(S).max()
    assert np.abs(u1 - u2).max() < 1e-14


def test_light_cone_window_matches_full_run():
    """The windowed evaluation used at full lattice sizes returns the same
    values as running the whole lattice."""
    rng = np.random.default_rng(26)
    shape = (14, 13, 15)
    flags = inputs.random_flags(15, 13, 14, 0.1, 27)
    rho = 1 + 1e-3 * rng.standard_normal(shape)
    u = 0.02 * rng.standard_normal((3,) + shape)
    F = (1e-5, 0, -2e-5)
    n = 4
    S = oracle.run(oracle.init(shape, rho, u, flags), 0.6, n, F=F, flags=flags)
    r, uu = oracle.macros(S, F=F, flags=flags)
    centres = [(0, 0, 0), (7, 6, 7), (13, 12, 14), (3, 11, 1)]
    rw, uw = oracle.run_window(rho, u, flags, 0.6, n, centres, F=F)
    for k, (z, y, x) in enumerate(centres):
        assert rw[k] == r[z, y, x]
        assert np.array_equal(uw[k], uu[:, z, y, x])

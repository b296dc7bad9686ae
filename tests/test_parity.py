"""GPU parity of the HIP path against the FP64 oracle (needs an MI355X).

Every comparison runs the same seeded inputs through the C ABI and through
the oracle.  Bounds: relative L2 error of the velocity over fluid sites
<= 1e-5 for FP32 storage and <= 2e-3 for FP16 storage; bit-exact results
where the method is a pure permutation (omega = 0) or a fixed point (rest).
"""
import math

import os

import numpy as np
import pytest

import oracle
import paper_2409_16781_amd as lbm
from paper_2409_16781_amd import inputs
from gpu_util import (FP64_SUM_TOL, TOL_U_BF16, bf16_bound, decode_raw, exact_state_totals, fluid_mask, gpu_run,
                      make_lattice, max_abs, oracle_run, rel_l2_u, require_gpu, say, streamed_pair, totals_gap_bound)

pytestmark = pytest.mark.gpu

TOL_U = {"f32": 1e-5, "f16": 2e-3}
VARIANTS = [0, 1, 2, 3]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    require_gpu()
    oracle.build(force=False)


# ------------------------------------------------------------ Taylor-Green --

@pytest.fixture(scope="module")
def tgv32_ref():
    cfg = inputs.tgv_box(32, u0=0.01, tau=0.8, steps=200)
    r, u, _ = oracle_run(cfg, 200)
    return cfg, r, u


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_tgv32_parity(tgv32_ref, codec, variant):
    cfg, r_ref, u_ref = tgv32_ref
    r, u, lat = gpu_run(cfg, 200, codec=codec, variant=variant)
    assert lat.info["variant"] == variant
    m = fluid_mask(cfg)
    err = rel_l2_u(u, u_ref, m)
    say(f"  rel-L2(u) = {err:.3e}  max|drho| = {max_abs(r, r_ref, m):.3e}")
    assert err <= TOL_U[codec]
    assert max_abs(r, r_ref, m) < (1e-6 if codec == "f32" else 1e-4)


def test_tgv32_bf16_bound(tgv32_ref):
    cfg, r_ref, u_ref = tgv32_ref
    r, u, _ = gpu_run(cfg, 200, codec="bf16")
    err = rel_l2_u(u, u_ref, fluid_mask(cfg))
    say(f"  BF16 rel-L2(u) = {err:.3e} (bound {TOL_U_BF16:g})")
    bf16_bound(err)


# --------------------------------------------- channel, porous, ragged sizes --

def _channel_small():
    cfg = inputs.channel(64, 32, 16, tau=0.6, g=1e-5, steps=300, noise=1e-4, seed=1)
    return cfg


def _porous(nx, ny, nz, frac, seed, tau=0.7, g=2e-5):
    rng = np.random.default_rng(seed)
    flags = inputs.random_flags(nx, ny, nz, frac, seed)
    rho = 1.0 + inputs.uniform_noise((nz, ny, nx), 1e-4, seed + 1)
    u = inputs.uniform_noise((3, nz, ny, nx), 1e-3, seed + 2)
    return dict(name=f"porous{nx}x{ny}x{nz}", shape=(nz, ny, nx), rho=rho, u=u, flags=flags, tau=tau,
                force=(g, -0.5 * g, 0.25 * g))


@pytest.mark.parametrize("variant", VARIANTS)
def test_channel_walls_force_parity(variant):
    cfg = _channel_small()
    r_ref, u_ref, _ = oracle_run(cfg, 300)
    r, u, _ = gpu_run(cfg, 300, variant=variant)
    m = fluid_mask(cfg)
    err = rel_l2_u(u, u_ref, m)
    say(f"  rel-L2(u) = {err:.3e}")
    assert err <= 1e-5
    assert np.all(r[~m] == 0) and np.all(u[:, ~m] == 0)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_porous_parity(codec, variant):
    cfg = _porous(48, 20, 12, 0.15, 31)
    steps = 60
    r_ref, u_ref, _ = oracle_run(cfg, steps)
    r, u, _ = gpu_run(cfg, steps, codec=codec, variant=variant)
    m = fluid_mask(cfg)
    err = rel_l2_u(u, u_ref, m)
    say(f"  rel-L2(u) = {err:.3e}")
    assert err <= TOL_U[codec]


@pytest.mark.parametrize("shape", [(9, 11, 37), (5, 7, 6), (3, 5, 66), (1, 1, 1), (2, 3, 130)])
@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_ragged_shapes_parity(shape, codec):
    nz, ny, nx = shape
    cfg = _porous(nx, ny, nz, 0.1 if nx * ny * nz > 8 else 0.0, 40 + nx)
    r_ref, u_ref, _ = oracle_run(cfg, 12)
    r, u, lat = gpu_run(cfg, 12, codec=codec)
    m = fluid_mask(cfg)
    err = rel_l2_u(u, u_ref, m)
    say(f"  {shape} variant={lat.info['variant']} rel-L2(u) = {err:.3e}")
    assert err <= TOL_U[codec]


# ------------------------------------------------------- bit-exact cases ----

def _random_raw(shape, codec, seed):
    rng = np.random.default_rng(seed)
    if codec == "f32":
        return rng.uniform(-1e-2, 1e-2, (19,) + shape).astype(np.float32)
    vals = rng.uniform(-1e-2, 1e-2, (19,) + shape)
    if codec == "f16":
        return vals.astype(np.float16).view(np.uint16)
    f32 = vals.astype(np.float32).view(np.uint32)
    return (f32 >> 16).astype(np.uint16)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("codec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(6, 10, 32), (3, 4, 512), (2, 3, 1536)])
def test_pure_streaming_bit_exact(codec, variant, walls, shape):
    """omega = 0 (tau = inf), F = 0: three steps permute the stored values;
    the GPU result equals the oracle's permutation of the same values exactly.
    At nx = 512 and 1536 every wave of the vector-row kernels lies inside one
    row (the kernels with wave-uniform row addressing); at nx = 32 a wave
    spans several rows."""
    nz, ny, nx = shape
    flags = inputs.random_flags(nx, ny, nz, 0.2, 51) if walls else None
    raw = _random_raw(shape, codec, 52)
    g = lbm.decode_state(raw, codec)
    with_variant = dict(name="omega0", shape=shape, tau=math.inf, flags=flags)
    lat = make_lattice(with_variant, codec, variant)
    lat.set_f(raw)
    lat.step(3)
    out, ref = streamed_pair(lbm.decode_state(lat.get_f(), codec), g, 3, flags)
    m = np.ones(shape, bool) if flags is None else flags == 0
    assert np.array_equal(out[:, m], ref[:, m])


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("codec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(16, 24, 8), (5, 6, 512)])
def test_sparse_solids_streaming_bit_exact(shape, codec, variant):
    """omega = 0 with a few isolated solid sites and part of one row solid:
    most waves hold no solid site and no bounce-back and read no masks; the
    waves around the solids (many rows per wave at nx = 8, half a row per
    wave at nx = 512, neighbours across wave seams and the periodic wrap)
    bounce back exactly like the oracle."""
    nz, ny, nx = shape
    flags = np.zeros(shape, np.uint8)
    flags[nz // 2, ny // 2, nx // 2] = 1
    flags[1, 0, 0] = 1
    flags[nz - 1, ny - 1, nx - 1] = 1
    flags[2, 3, : max(1, nx // 3)] = 1
    raw = _random_raw(shape, codec, 53)
    g = lbm.decode_state(raw, codec)
    lat = make_lattice(dict(name="sparse", shape=shape, tau=math.inf, flags=flags), codec, variant)
    lat.set_f(raw)
    lat.step(3)
    out, ref = streamed_pair(lbm.decode_state(lat.get_f(), codec), g, 3, flags)
    m = flags == 0
    assert np.array_equal(out[:, m], ref[:, m])


@pytest.mark.parametrize("codec", ["f32", "f16", "bf16"])
def test_rest_state_is_exactly_invariant(codec):
    cfg = dict(name="rest", shape=(8, 12, 16), tau=0.7, flags=inputs.channel_flags(16, 12, 8))
    lat = make_lattice(cfg, codec)
    lat.step(70)
    raw = lat.get_f()
    assert not np.any(raw)


# ---------------------------------------------------- same-pass macros -----

@pytest.mark.parametrize("variant", VARIANTS)
def test_same_pass_macros_match_state_macros_and_oracle(variant):
    cfg = _porous(32, 12, 10, 0.1, 61)
    steps = 25
    r1, u1, lat = gpu_run(cfg, steps, variant=variant, same_pass=True)
    r2, u2 = lat.macros()
    r2, u2 = r2.double().cpu().numpy(), u2.double().cpu().numpy()
    m = fluid_mask(cfg)
    assert max_abs(r1, r2, m) < 2e-7
    assert np.abs(u1 - u2).max() < 1e-8
    assert np.all(r1[~m] == 0) and np.all(u1[:, ~m] == 0)
    r_ref, u_ref, _ = oracle_run(cfg, steps)
    assert rel_l2_u(u1, u_ref, m) <= 1e-5


# ------------------------------------------------------- FP64 totals -------

def test_conservation_totals_match_oracle_and_reproduce():
    cfg = _porous(40, 16, 12, 0.1, 71)
    steps = 40
    lat = make_lattice(cfg)
    m = fluid_mask(cfg)
    S = oracle.init(cfg["shape"], cfg["rho"], cfg["u"], cfg["flags"])
    for t in range(steps):
        lat.step(1)
        S = oracle.run(S, cfg["tau"], 1, F=cfg["force"], flags=cfg["flags"])
        ref = oracle.sums(S, cfg["flags"])
        tot = lat.sums(1)[0]
        g = decode_raw(lat.get_f(), "f32")
        # the totals are the FP64 sums of the stored state ...
        exact, scale = exact_state_totals(g, m)
        assert np.all(np.abs(tot - exact) <= FP64_SUM_TOL * scale), (t, tot, exact)
        # ... so they differ from the oracle's by the summed state difference
        # only (FP32 storage and FP32 arithmetic of the GPU state)
        bound = totals_gap_bound(g, S, m)
        assert np.all(np.abs(tot - ref) <= bound), (t, tot - ref, bound)
    sums = lat.sums(steps)
    lat2 = make_lattice(cfg)
    lat2.step(steps)
    assert np.array_equal(lat2.sums(steps), sums)


@pytest.mark.parametrize("codec", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(12, 16, 40), (64, 64, 64), (128, 128, 128)])
def test_totals_are_fp64_sums_of_the_stored_state(codec, shape):
    """The per-step totals equal the sums of the stored values (read back
    raw, summed in extended precision) to FP64 rounding, also
    on lattices with more than one chunk of workgroup partials (128^3 has
    2048 step workgroups), and a run of n steps appends the same totals as n
    single steps."""
    nz, ny, nx = shape
    cfg = _porous(nx, ny, nz, 0.05, 91) if nx == 40 else dict(
        name=f"smooth{nx}", shape=shape, tau=0.6, force=(1e-5, 0.0, 0.0),
        rho=1.0 + inputs.uniform_noise(shape, 1e-3, 92), u=inputs.uniform_noise((3,) + shape, 2e-2, 93))
    a = make_lattice(cfg, codec)
    a.step(7)
    tot = a.sums(7)
    exact, scale = exact_state_totals(decode_raw(a.get_f(), codec), fluid_mask(cfg))
    err = np.abs(tot[-1] - exact)
    say(f"  {codec} {shape}: |totals - extended-precision sums of the stored state| = {err}, "
        f"bound {FP64_SUM_TOL * scale}")
    assert np.all(err <= FP64_SUM_TOL * scale)
    b = make_lattice(cfg, codec)
    for _ in range(7):
        b.step(1)
    assert np.array_equal(b.sums(7), tot)
    a.close()
    b.close()


def test_mass_is_conserved_to_fp32_storage_rounding():
    cfg = _porous(40, 16, 12, 0.1, 72)
    lat = make_lattice(cfg)
    lat.step(200)
    s = lat.sums(200)
    drift = abs(s[-1, 0] - s[0, 0]) / s[0, 0]
    say(f"  relative mass drift over 200 steps: {drift:.2e}")
    assert drift < 1e-9


def test_nan_in_state_is_reported_unstable():
    cfg = dict(name="nan", shape=(4, 8, 16), tau=0.8)
    lat = make_lattice(cfg)
    raw = lat.get_f()
    raw[3, 1, 2, 5] = np.nan
    lat.set_f(raw)
    lat.step(2)
    with pytest.raises(lbm.LBError) as ei:
        lat.sums(1)
    assert ei.value.code == lbm.LB_EUNSTABLE


# ----------------------------------------------- graphs and checkpoints ----

@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_graph_replay_equals_eager_steps(codec):
    cfg = _porous(32, 10, 8, 0.1, 81)
    a = make_lattice(cfg, codec)
    a.step(131)          # one captured run of 131 steps (odd: ends on the other array)
    for _ in range(3):   # a run of 65 steps captured from each parity, replayed alternately
        a.step(65)
    a.step(2100)         # two replays of a 1024-step run and an eager tail
    total = 131 + 3 * 65 + 2100
    b = make_lattice(cfg, codec)
    for _ in range(total):
        b.step(1)
    assert np.array_equal(a.get_f(), b.get_f())
    assert np.array_equal(a.sums(total), b.sums(total))


def test_chained_totals_equal_per_step_reduce_on_many_chunks():
    """128^3 runs 2048 step workgroups, i.e. eight chunks of the totals reduce:
    a run of 70 steps (graph replays whose steps append the previous step's
    totals) gives the same state and the same ring, bit for bit, as 70 single
    steps each closed by its own totals kernel."""
    cfg = inputs.tgv_noise_box(128, u0=0.01, tau=0.55, steps=70, noise=1e-3, seed=2)
    a = make_lattice(cfg, "f32")
    assert a.info["grid"] > 8 * 256 - 1
    say(f"[gpu] chained totals 128^3 grid={a.info['grid']}")
    a.step(70)
    b = make_lattice(cfg, "f32")
    for _ in range(70):
        b.step(1)
    assert np.array_equal(a.get_f(), b.get_f())
    assert np.array_equal(a.sums(70).view(np.uint64), b.sums(70).view(np.uint64))
    a.close()
    b.close()


@pytest.mark.parametrize("codec", ["f32", "f16", "s16"])
def test_tune_keeps_the_state_and_picks_a_valid_shape(codec):
    """lb_tune times launch shapes with launches that read the current state
    and write the other array: state, step count and totals are unchanged,
    and the lattice then steps on in the chosen shape within the bound."""
    cfg = inputs.channel(64, 34, 16, tau=0.6, g=1e-5, steps=50, noise=1e-4, seed=1)
    lat = make_lattice(cfg, codec)
    lat.step(7)
    raw, tot = lat.get_f(), lat.sums(7)
    info = lat.tune(5)
    say(f"  {codec}: tuned shape variant={info['variant']} tile_order={info['tile_order']} grid={info['grid']}")
    assert info["variant"] in (1, 2, 3) and info["tile_order"] in (0, 1, 2) and info["pull_nt"] in (0, 1)
    assert np.array_equal(lat.get_f(), raw) and np.array_equal(lat.sums(7), tot) and lat.steps_done == 7
    lat.step(43)
    _, u = lat.macros()
    _, u_ref, _ = oracle_run(cfg, 50)
    err = rel_l2_u(u.double().cpu().numpy(), u_ref, fluid_mask(cfg))
    assert err <= (1e-5 if codec == "f32" else 2e-3), err
    lat.close()


@pytest.mark.parametrize("codec,variant", [("f32", 1), ("f32", 3), ("f16", 2)])
def test_tile_orders_give_the_same_state(codec, variant):
    """Tile orders 0 (linear), 1 (a contiguous range per XCD) and 2 (blocks
    of 64 tiles rotated) map workgroups to tiles by bijections: the same
    state bit for bit, and totals equal up to the order of the FP64 sum.
    The lattice has a partial last block of tiles."""
    cfg = _porous(64, 36, 30, 0.1, 29)
    lats = []
    for order in ("0", "1", "2"):
        old = os.environ.get("LB_TILE_ORDER")
        os.environ["LB_TILE_ORDER"] = order
        try:
            lat = make_lattice(cfg, codec, variant)
        finally:
            if old is None:
                os.environ.pop("LB_TILE_ORDER", None)
            else:
                os.environ["LB_TILE_ORDER"] = old
        assert lat.info["tile_order"] == int(order) and lat.info["variant"] == variant
        say(f"[gpu] tile order {order} {codec} variant={variant} grid={lat.info['grid']}")
        lat.step(3)
        lat.step(70)
        lats.append(lat)
    ref = lats[0].get_f()
    tot = lats[0].sums(73)
    for lat in lats[1:]:
        assert np.array_equal(lat.get_f(), ref)
        assert np.allclose(lat.sums(73), tot, rtol=1e-12, atol=1e-12)
    for lat in lats:
        lat.close()


@pytest.mark.parametrize("codec,variant", [("f32", 1), ("f32", 3), ("f16", 2), ("bf16", 1), ("s16", 2), ("s16", 3)])
def test_pull_cache_policy_changes_no_bits(codec, variant):
    """Lattices with solids pull with cached or with non-temporal loads
    (LB_PULL_NT, a dimension of lb_tune): the same state and totals, bit for
    bit, over single steps and a captured run."""
    cfg = _porous(64, 20, 12, 0.15, 23)
    lats = []
    for nt in ("0", "1"):
        old = os.environ.get("LB_PULL_NT")
        os.environ["LB_PULL_NT"] = nt
        try:
            lat = make_lattice(cfg, codec, variant)
        finally:
            if old is None:
                os.environ.pop("LB_PULL_NT", None)
            else:
                os.environ["LB_PULL_NT"] = old
        assert lat.info["pull_nt"] == int(nt) and lat.info["variant"] == variant
        say(f"[gpu] pull policy nt={nt} {codec} variant={variant}")
        for _ in range(3):
            lat.step(1)
        lat.step(70)
        lats.append(lat)
    a, b = lats
    assert np.array_equal(a.get_f(), b.get_f())
    assert np.array_equal(a.sums(73).view(np.uint64), b.sums(73).view(np.uint64))
    a.close()
    b.close()


@pytest.mark.parametrize("codec", ["f32", "f16", "bf16"])
def test_checkpoint_resume_is_bit_exact(codec):
    cfg = _porous(32, 12, 8, 0.1, 91)
    n = 37
    a = make_lattice(cfg, codec)
    a.step(2 * n)
    b = make_lattice(cfg, codec)
    b.step(n)
    saved = b.get_f()
    b.close()
    c = make_lattice(dict(cfg, rho=None, u=None), codec)
    c.set_f(saved)
    c.step(n)
    assert np.array_equal(a.get_f(), c.get_f())
    assert np.array_equal(a.sums(1), c.sums(1))


def test_errors_on_device():
    require_gpu()
    with pytest.raises(lbm.LBError):
        lbm.Lattice(8, 8, 8, 0.5)
    # rows so long that one storage block would reach 1 GiB: refused before
    # anything is allocated (the kernels' in-block offsets are 32-bit)
    with pytest.raises(lbm.LBError, match="storage block"):
        lbm.Lattice(1 << 24, 1, 1, 0.8)
    lat = lbm.Lattice(8, 8, 8, 0.8)
    with pytest.raises(lbm.LBError):
        lat.sums(1)        # no steps yet
    with pytest.raises(lbm.LBError):
        lat.step(-1)
    lat.step(0)
    assert lat.steps_done == 0

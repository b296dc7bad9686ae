"""Scaled 16-bit fixed-point storage (codec "s16", LB_S16) through the C ABI.

* Parity with the FP64 oracle under the 16-bit bound (rel-L2(u) <= 2e-3) on
  the Taylor-Green box, a porous lattice with forces and ragged shapes, for
  every kernel variant; on the Taylor-Green box the error is also below
  FP16 storage's (finer steps than FP16 at the largest values).
* omega = 0 permutations and the rest state, bit for bit (decode and encode
  are exact on the code grid).
* The per-step totals are the FP64 sums of the stored codes.
* Graph replay = single steps, checkpoint/resume (codes plus exponents).
* Overflow: a channel started from rest has ranges sized by its density
  noise; as the flow develops, codes leave their range, the flagged steps are
  redone with wider ranges, and the result still meets the bound.
* A run that blows up ends in LB_EUNSTABLE; the codec is refused where it is
  not supported.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
import paper_2409_16781_amd as lbm
from paper_2409_16781_amd import inputs
from gpu_util import (FP64_SUM_TOL, decode_raw, exact_state_totals, fluid_mask, gpu_run, make_lattice, oracle_run,
                      rel_l2_u, require_gpu, say, streamed_pair)

pytestmark = pytest.mark.gpu

TOL = 2e-3
VARIANTS = [0, 1, 2, 3]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    require_gpu()
    oracle.build(force=False)


def _porous(nx, ny, nz, frac, seed, tau=0.7, g=2e-5):
    flags = inputs.random_flags(nx, ny, nz, frac, seed)
    rho = 1.0 + inputs.uniform_noise((nz, ny, nx), 1e-4, seed + 1)
    u = inputs.uniform_noise((3, nz, ny, nx), 1e-3, seed + 2)
    return dict(name=f"porous{nx}x{ny}x{nz}", shape=(nz, ny, nx), rho=rho, u=u, flags=flags, tau=tau,
                force=(g, -0.5 * g, 0.25 * g))


@pytest.fixture(scope="module")
def tgv32_ref():
    cfg = inputs.tgv_box(32, u0=0.01, tau=0.8, steps=200)
    r, u, _ = oracle_run(cfg, 200)
    return cfg, r, u


@pytest.mark.parametrize("variant", VARIANTS)
def test_tgv32_parity_and_finer_than_fp16(tgv32_ref, variant):
    cfg, r_ref, u_ref = tgv32_ref
    m = fluid_mask(cfg)
    _, u, lat = gpu_run(cfg, 200, codec="s16", variant=variant)
    assert lat.info["variant"] == variant and lat.info["codec"] == lbm.LB_S16
    err = rel_l2_u(u, u_ref, m)
    _, u16, _ = gpu_run(cfg, 200, codec="f16", variant=variant)
    err16 = rel_l2_u(u16, u_ref, m)
    say(f"  s16 rel-L2(u) = {err:.3e} (f16 {err16:.3e}), exponents {lat.get_scales()}, "
        f"widenings {lat.info['rescales']}")
    assert err <= TOL
    assert err < err16


@pytest.mark.parametrize("variant", VARIANTS)
def test_porous_parity(variant):
    cfg = _porous(48, 20, 12, 0.15, 31)
    r_ref, u_ref, _ = oracle_run(cfg, 60)
    _, u, lat = gpu_run(cfg, 60, codec="s16", variant=variant)
    err = rel_l2_u(u, u_ref, fluid_mask(cfg))
    say(f"  rel-L2(u) = {err:.3e}, widenings {lat.info['rescales']}")
    assert err <= TOL


@pytest.mark.parametrize("shape", [(9, 11, 37), (5, 7, 6), (3, 5, 66), (1, 1, 1), (2, 3, 130)])
def test_ragged_shapes_parity(shape):
    nz, ny, nx = shape
    cfg = _porous(nx, ny, nz, 0.1 if nx * ny * nz > 8 else 0.0, 40 + nx)
    _, u_ref, _ = oracle_run(cfg, 12)
    _, u, lat = gpu_run(cfg, 12, codec="s16")
    err = rel_l2_u(u, u_ref, fluid_mask(cfg))
    say(f"  {shape} variant={lat.info['variant']} rel-L2(u) = {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(6, 10, 32), (3, 4, 512)])
def test_pure_streaming_bit_exact(variant, walls, shape):
    """omega = 0, F = 0: three steps permute the stored codes exactly (at
    nx = 512 with wave-uniform row addressing)."""
    nz, ny, nx = shape
    flags = inputs.random_flags(nx, ny, nz, 0.2, 51) if walls else None
    lat = make_lattice(dict(name="omega0", shape=shape, tau=math.inf, flags=flags), "s16", variant)
    exps = lat.get_scales()
    raw = np.random.default_rng(52).integers(-30000, 30000, (19,) + shape).astype(np.int16).view(np.uint16)
    if flags is not None:
        raw[:, flags == 1] = 0
    lat.set_f(raw)
    lat.step(3)
    out, ref = streamed_pair(lbm.decode_state(lat.get_f(), "s16", exps), lbm.decode_state(raw, "s16", exps), 3, flags)
    m = np.ones(shape, bool) if flags is None else flags == 0
    assert np.array_equal(out[:, m], ref[:, m])
    assert lat.info["rescales"] == 0


def test_rest_state_is_exactly_invariant():
    cfg = dict(name="rest", shape=(8, 12, 16), tau=0.7, flags=inputs.channel_flags(16, 12, 8))
    lat = make_lattice(cfg, "s16")
    lat.step(70)
    assert not np.any(lat.get_f())


@pytest.mark.parametrize("shape", [(12, 16, 40), (64, 64, 64)])
def test_totals_are_fp64_sums_of_the_stored_codes(shape):
    nz, ny, nx = shape
    cfg = _porous(nx, ny, nz, 0.05, 91)
    a = make_lattice(cfg, "s16")
    a.step(9)
    tot = a.sums(9)
    exact, scale = exact_state_totals(decode_raw(a.get_f(), "s16", a.get_scales()), fluid_mask(cfg))
    assert np.all(np.abs(tot[-1] - exact) <= FP64_SUM_TOL * scale), (tot[-1], exact)


def test_graph_replay_equals_single_steps():
    cfg = _porous(32, 10, 8, 0.1, 81)
    a = make_lattice(cfg, "s16")
    a.step(131)
    b = make_lattice(cfg, "s16")
    for _ in range(131):
        b.step(1)
    assert np.array_equal(a.get_scales(), b.get_scales())
    assert np.array_equal(a.get_f(), b.get_f())
    assert np.array_equal(a.sums(131), b.sums(131))


def test_checkpoint_resume_is_bit_exact():
    cfg = _porous(32, 10, 8, 0.1, 82)
    a = make_lattice(cfg, "s16")
    a.step(40)
    raw, exps = a.get_f(), a.get_scales()
    a.step(30)
    b = make_lattice(dict(cfg, rho=None, u=None), "s16")
    b.set_scales(exps)
    b.set_f(raw)
    b.step(30)
    assert np.array_equal(a.get_f(), b.get_f())


def test_overflowing_steps_are_redone_with_wider_ranges():
    """From rest (density noise 1e-4 only) the ranges are sized for the noise;
    the force accelerates the flow by two orders of magnitude, so codes leave
    their ranges several times.  Each time the flagged step and those after
    it are redone with ranges one bit wider; the result meets the bound."""
    cfg = inputs.channel(32, 34, 8, tau=0.6, g=2e-5, steps=400, noise=1e-4, seed=1)
    _, u_ref, _ = oracle_run(cfg, 400)
    lat = make_lattice(cfg, "s16")
    e0 = lat.get_scales()
    lat.step(400)           # one captured run of 400 steps
    r, u = lat.macros()
    e1 = lat.get_scales()
    err = rel_l2_u(u.double().cpu().numpy(), u_ref, fluid_mask(cfg))
    say(f"  exponents {e0} -> {e1}, widenings {lat.info['rescales']}, rel-L2(u) = {err:.3e}")
    assert lat.info["rescales"] >= 2
    # each widening moves at least one weight class by one bit, none narrows
    assert np.all(e1 <= e0) and (e0 - e1).sum() >= lat.info["rescales"]
    assert lat.steps_done == 400
    assert err <= TOL
    s = lat.sums(400)       # one totals entry per step, none lost to the redone steps
    assert np.all(np.isfinite(s))
    assert abs(s[-1, 0] - s[0, 0]) <= 1e-6 * s[0, 0]


def test_same_pass_macros_are_those_of_the_settled_state():
    cfg = inputs.channel(32, 34, 8, tau=0.6, g=2e-5, steps=200, noise=1e-4, seed=1)
    lat = make_lattice(cfg, "s16")
    r1, u1 = lat.step_macros(200)
    r2, u2 = lat.macros()
    assert lat.info["rescales"] >= 1
    assert np.array_equal(u1.cpu().numpy(), u2.cpu().numpy())
    assert np.array_equal(r1.cpu().numpy(), r2.cpu().numpy())


def test_blow_up_is_reported_unstable():
    """tau close to 1/2 with a large initial velocity: the run blows up; the
    ranges widen until the widest, then the lattice reports LB_EUNSTABLE."""
    shape = (8, 8, 16)
    u = inputs.uniform_noise((3,) + shape, 0.35, 7)
    cfg = dict(name="blowup", shape=shape, tau=0.5001, rho=np.ones(shape), u=u)
    lat = make_lattice(cfg, "s16")
    lat.step(400)
    with pytest.raises(lbm.LBError) as exc:
        lat.sync()
    assert exc.value.code == lbm.LB_EUNSTABLE


def test_codec_refused_where_unsupported():
    L = lbm.lib()
    assert not L.lb_create_ex(16, 8, 4, 0.7, None, lbm.LB_S16 | lbm.LB_INPLACE, None)
    assert "LB_INPLACE" in lbm.last_error()
    dims = (ctypes.c_int * 3)(8, 8, 8)
    taus = (ctypes.c_double * 1)(0.7)
    assert not L.lb_batch_create(1, dims, taus, None, lbm.LB_S16, None, 0)
    assert "batches" in lbm.last_error()
    lat = make_lattice(dict(name="s", shape=(4, 6, 8), tau=0.7), "s16")
    J = ctypes.c_double(0.0)
    assert L.lb_outlet_flux(lat.handle, ctypes.byref(J)) == lbm.LB_EINVAL
    f32 = make_lattice(dict(name="f", shape=(4, 6, 8), tau=0.7), "f32")
    assert L.lb_get_scales(f32.handle, (ctypes.c_int * 3)()) == lbm.LB_EINVAL
    bad = (ctypes.c_int * 3)(3, 20, 20)
    assert L.lb_set_scales(lat.handle, bad) == lbm.LB_EINVAL

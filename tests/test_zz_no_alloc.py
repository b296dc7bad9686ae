"""lb_step_noalloc (the allocation-free variant of lb_step) against lb_step,
through the C ABI: two calls in a row, the second on a smaller lattice, each
checked bit for bit (state and per-step FP64 totals) against lb_step on an
identically initialised lattice, and the first also against the FP64 oracle.
The two entry points run the same kernels; only where the totals' scratch
lives differs, so equality is exact."""
import ctypes

import numpy as np
import pytest

import paper_2409_16781_amd as lbm
from paper_2409_16781_amd import inputs

from gpu_util import fluid_mask, kernel_variant, make_lattice, oracle_run, rel_l2_u, require_gpu, say

pytestmark = pytest.mark.gpu


def _pair(cfg, codec):
    return make_lattice(cfg, codec), make_lattice(cfg, codec)


def _compare(ref, lat, steps):
    ref.sync()
    lat.sync()
    a, b = ref.get_f(), lat.get_f()
    assert a.dtype == b.dtype and a.shape == b.shape
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), "state differs from lb_step's"
    ta, tb = ref.sums(steps), lat.sums(steps)
    assert np.array_equal(ta.view(np.uint64), tb.view(np.uint64)), (ta[-1], tb[-1])
    assert ref.steps_done == lat.steps_done == steps


def test_noalloc_matches_step_on_two_calls_in_a_row():
    require_gpu()
    L = lbm.lib()
    # call 1: 48^3 Taylor-Green + noise, FP32, all fluid, 37 steps (odd: ends on the other array)
    big = inputs.tgv_noise_box(48, u0=0.01, tau=0.55, steps=37, noise=1e-3, seed=2)
    # call 2: a smaller walled channel with a body force, FP16 storage, 12 steps
    small = inputs.channel(24, 20, 16, tau=0.6, g=1e-5, steps=12, noise=1e-4, seed=1)
    with kernel_variant(None):
        ref1, lat1 = _pair(big, "f32")
        ref2, lat2 = _pair(small, "f16")
    say(f"[gpu] noalloc call 1: {big['shape']} f32 grid={lat1.info['grid']}")
    assert L.lb_step_noalloc(lat1.handle, 37) == lbm.LB_OK, lbm.last_error()
    say(f"[gpu] noalloc call 2: {small['shape']} f16 grid={lat2.info['grid']}")
    assert L.lb_step_noalloc(lat2.handle, 12) == lbm.LB_OK, lbm.last_error()
    assert L.lb_step_noalloc(lat2.handle, 0) == lbm.LB_OK  # no-op
    ref1.step(37)
    ref2.step(12)
    _compare(ref1, lat1, 37)
    _compare(ref2, lat2, 12)
    # the first call's result also against the oracle (FP32 bound)
    _, u, _ = oracle_run(big, 37)
    _, ug = lat1.macros()
    err = rel_l2_u(ug.double().cpu().numpy(), u, fluid_mask(big))
    assert err <= 1e-5, err
    for h in (ref1, lat1, ref2, lat2):
        h.close()


def test_noalloc_continues_a_run_of_lb_step():
    """Mixed use on one lattice: lb_step, then lb_step_noalloc, then lb_step
    again, equals lb_step alone (the totals ring stays in step order)."""
    require_gpu()
    cfg = inputs.channel(32, 18, 10, tau=0.7, g=1e-5, steps=0, noise=1e-4, seed=5)
    with kernel_variant(None):
        ref, lat = _pair(cfg, "f32")
    say(f"[gpu] noalloc mixed run {cfg['shape']}")
    ref.step(70)
    lat.step(5)
    assert lbm.lib().lb_step_noalloc(lat.handle, 33) == lbm.LB_OK, lbm.last_error()
    lat.step(32)
    _compare(ref, lat, 70)
    ref.close()
    lat.close()


def test_noalloc_rejects_lattices_beyond_the_scratch():
    """One site per lane (odd nx) on 257 x 512 x 260 sites needs 133 640 step
    workgroups, more than the static scratch holds: a clear error, no launch."""
    require_gpu()
    with kernel_variant(None):
        lat = lbm.Lattice(257, 512, 260, 0.8, codec="f16")
    assert lat.info["grid"] > 131072
    say(f"[gpu] noalloc oversize grid={lat.info['grid']}")
    rc = lbm.lib().lb_step_noalloc(lat.handle, 1)
    assert rc == lbm.LB_EINVAL
    assert "scratch" in lbm.last_error()
    assert lat.steps_done == 0
    lat.close()


def test_noalloc_rejects_bad_arguments():
    require_gpu()
    assert lbm.lib().lb_step_noalloc(ctypes.c_void_p(0), 1) == lbm.LB_ESTATE
    cfg = inputs.tgv_box(8, 0.01, 0.8, 0)
    lat = make_lattice(cfg)
    assert lbm.lib().lb_step_noalloc(lat.handle, -1) == lbm.LB_EINVAL
    lat.close()

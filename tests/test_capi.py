"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/lb.h declares, and rejects bad arguments before touching HIP."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2409_16781_amd as lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb(?:2d)?_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lb_create", "lb_step", "lb_macros", "lb_destroy", "lb_init_eq", "lb_sums",
                     "lb_get_f", "lb_set_f", "lb_set_force", "lb_create_ex", "lb_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    assert sorted(lbm._SIGNATURES) == declared_functions()
    assert "lb2d_create" in declared_functions()


@pytest.mark.parametrize("args,needle", [
    ((0, 8, 0.8, None, 0.0, 0.0), "extents"),
    ((8, 8, 0.5, None, 0.0, 0.0), "tau"),
    ((8, 8, float("nan"), None, 0.0, 0.0), "tau"),
    ((8, 8, 0.8, None, float("inf"), 0.0), "lid"),
    ((1 << 16, 1 << 15, 0.8, None, 0.0, 0.0), "extents"),
])
def test_create2d_rejects_bad_arguments(args, needle):
    h = lbm.lib().lb2d_create(*args, None)
    assert not h
    assert needle in lbm.last_error()


def test_create2d_rejects_bad_flags():
    flags = np.zeros((4, 4), dtype=np.uint8)
    flags[1, 2] = 3
    assert not lbm.lib().lb2d_create(4, 4, 0.8, flags.ctypes.data_as(ctypes.c_void_p), 0.0, 0.0, None)
    assert "flag value 3" in lbm.last_error()


def test_d2q9_calls_reject_null_handles():
    L = lbm.lib()
    assert L.lb2d_step(None, 1) == lbm.LB_ESTATE
    assert L.lb2d_sync(None) == lbm.LB_ESTATE
    L.lb2d_destroy(None)


@pytest.mark.parametrize("args,needle", [
    ((0, 4, 4, 0.8), "extents"),
    ((4, -1, 4, 0.8), "extents"),
    ((4, 4, 4, 0.5), "tau"),
    ((4, 4, 4, 0.3), "tau"),
    ((4, 4, 4, float("nan")), "tau"),
    ((1 << 11, 1 << 10, 1 << 10, 0.8), "exceeds"),
])
def test_create_rejects_bad_arguments(args, needle):
    L = lbm.lib()
    h = L.lb_create(*args, None)
    assert not h
    assert needle in lbm.last_error()


def test_create_rejects_bad_codec_and_flags():
    L = lbm.lib()
    assert not L.lb_create_ex(4, 4, 4, 0.8, None, 7, None)
    assert "codec" in lbm.last_error()
    flags = np.zeros(64, dtype=np.uint8)
    flags[10] = 2
    assert not L.lb_create(4, 4, 4, 0.8, flags.ctypes.data_as(ctypes.c_void_p))
    assert "flag value 2" in lbm.last_error()


def test_null_handle_is_rejected_everywhere():
    L = lbm.lib()
    assert L.lb_step(None, 1) == lbm.LB_ESTATE
    assert L.lb_macros(None, None, None) == lbm.LB_ESTATE
    assert L.lb_set_force(None, 0.0, 0.0, 0.0) == lbm.LB_ESTATE
    assert L.lb_sync(None) == lbm.LB_ESTATE
    assert L.lb_steps_done(None) == -1
    assert L.lb_query(None, 0) == -1
    L.lb_destroy(None)  # no-op


def test_tau_infinity_is_accepted_by_validation():
    """tau = +inf (omega = 0) passes argument checks; without a GPU the call
    then fails on the device query, with a HIP error rather than EINVAL."""
    L = lbm.lib()
    h = L.lb_create(4, 4, 4, math.inf, None)
    if h:  # a GPU is present
        L.lb_destroy(h)
    else:
        assert "tau" not in lbm.last_error()


def _batch_create(dims, taus, flags=None, storage=0):
    L = lbm.lib()
    d = np.ascontiguousarray(np.array(dims, dtype=np.int32).reshape(-1))
    t = np.ascontiguousarray(np.array(taus, dtype=np.float64))
    return L.lb_batch_create(len(taus), d.ctypes.data_as(ctypes.c_void_p), t.ctypes.data_as(ctypes.c_void_p),
                             flags, storage, None, 0)


@pytest.mark.parametrize("dims,taus,needle", [
    ([(4, 4, 4), (0, 4, 4)], [0.8, 0.8], "extents"),
    ([(4, 4, 4), (4, 4, 4)], [0.8, 0.5], "tau"),
    ([(4, 4, 4)], [float("nan")], "tau"),
    ([(1 << 11, 1 << 10, 1 << 10)], [0.8], "too large"),
])
def test_batch_create_rejects_bad_arguments(dims, taus, needle):
    assert not _batch_create(dims, taus)
    assert needle in lbm.last_error()


def test_batch_create_rejects_bad_codec_and_count():
    assert not _batch_create([(4, 4, 4)], [0.8], storage=9)
    assert "codec" in lbm.last_error()
    L = lbm.lib()
    assert not L.lb_batch_create(0, None, None, None, 0, None, 0)
    assert "count" in lbm.last_error()


def test_batch_null_handle_is_rejected_everywhere():
    L = lbm.lib()
    assert L.lb_batch_step(None, 1) == lbm.LB_ESTATE
    assert L.lb_batch_macros(None, 0, None, None) == lbm.LB_ESTATE
    assert L.lb_batch_set_force(None, -1, 0.0, 0.0, 0.0) == lbm.LB_ESTATE
    assert L.lb_batch_sums(None, 0, None, 1) == lbm.LB_ESTATE
    assert L.lb_batch_sync(None) == lbm.LB_ESTATE
    assert L.lb_batch_steps_done(None) == -1
    assert L.lb_batch_query(None, 0) == -1
    L.lb_batch_destroy(None)  # no-op


def test_objective_entry_points_reject_a_null_handle():
    L = lbm.lib()
    J = ctypes.c_double(0.0)
    assert L.lb_outlet_flux(None, ctypes.byref(J)) == lbm.LB_ESTATE
    assert L.lb_grad_outlet_flux_x(None, 10, 5, None, None) == lbm.LB_ESTATE

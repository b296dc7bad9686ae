"""GPU adjoint (gradient of the outlet mass flux with respect to a per-site
x-force) against the FP64 oracle's adjoint, against finite differences of
the GPU's own forward model, and through torch.autograd (needs an MI355X).

Objective: J = sum of rho u_x over the fluid sites of the plane x = nx - 1
after n steps.  The oracle's adjoint is pinned on the CPU by central
differences (tests/test_oracle_adjoint.py).  Bound on the GPU gradient:
relative L2 error over fluid cells <= 1e-4 (FP32 states and FP32 adjoint
arithmetic; each step adds a relative rounding of order 1e-7 to the adjoint
state, and the gradient sums n steps of it).
"""
import json
import os

import numpy as np
import pytest

import oracle
import paper_2409_16781_amd as lbm
from paper_2409_16781_amd import inputs
from gpu_util import W19, kernel_variant, require_gpu, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL_GRAD = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _setup():
    require_gpu()
    oracle.build(force=False)


def small_case(nx=16, ny=12, nz=10, steps=60, seed=21):
    flags = inputs.sphere_flags(nx, ny, nz, 0.85, seed, rmin=1.5, rmax=2.5)
    rng = np.random.default_rng(seed + 1)
    rho = 1.0 + rng.uniform(-1e-4, 1e-4, (nz, ny, nx))
    fx = rng.uniform(0.0, 5e-7, (nz, ny, nx)).astype(np.float32) * (flags == 0)
    return dict(shape=(nz, ny, nx), flags=flags, rho=rho, u=np.zeros((3, nz, ny, nx)), tau=0.6,
                force=(1e-6, 0.0, 0.0), fx=fx.astype(np.float32), steps=steps)


def gpu_lattice(c, variant=None):
    torch = require_gpu()
    nz, ny, nx = c["shape"]
    with kernel_variant(variant):
        lat = lbm.Lattice(nx, ny, nz, c["tau"], flags=c["flags"])
    lat.set_force(*c["force"])
    lat.init_eq(torch.from_numpy(c["rho"]).cuda(), torch.from_numpy(c["u"]).cuda())
    lat.set_force_field(torch.from_numpy(c["fx"]).cuda())
    return lat


def gpu_gradient(c, every, variant=None):
    """dJ/dF_x of the outlet flux through lb_grad_outlet_flux_x (seed and
    direct term built by the library); J of the final state is checked to be
    the one lb_outlet_flux reports afterwards."""
    lat = gpu_lattice(c, variant)
    J, g = lat.grad_outlet_flux_x(c["steps"], every)
    assert J == lat.outlet_flux()
    return g.double().cpu().numpy(), lat


def test_generic_seed_entry_point_equals_the_outlet_objective():
    """lb_grad_force_x with the outlet seed written out here (c_ix at the
    outlet's fluid sites) plus the direct term -1/2 gives the same gradient
    as lb_grad_outlet_flux_x, bit for bit."""
    torch = require_gpu()
    c = small_case(steps=20)
    g_lib, l1 = gpu_gradient(c, every=6)
    l2 = gpu_lattice(c)
    fluid = torch.from_numpy(c["flags"] == 0).cuda()
    cx = torch.tensor([0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0], dtype=torch.float32,
                      device="cuda")
    seed = torch.zeros((19,) + c["shape"], dtype=torch.float32, device="cuda")
    seed[:, :, :, -1] = cx[:, None, None] * fluid[None, :, :, -1].float()
    g = l2.grad_force_x(c["steps"], 6, seed)
    g[:, :, -1] -= 0.5 * fluid[:, :, -1].float()
    assert np.array_equal(g.double().cpu().numpy(), g_lib)
    l1.close()
    l2.close()


def oracle_gradient(c, every=None):
    S0 = oracle.init(c["shape"], c["rho"], c["u"], c["flags"])
    return oracle.grad_outlet_flux(S0, c["tau"], c["steps"], F=c["force"], flags=c["flags"],
                                   Fx_field=c["fx"].astype(np.float64), every=every)


def rel_l2(a, b, m):
    d = (a - b)[m]
    return float(np.sqrt((d * d).sum() / (b[m] ** 2).sum()))


@pytest.fixture(scope="module")
def small_ref():
    c = small_case()
    J, g = oracle_gradient(c)
    return c, J, g


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_gradient_matches_oracle(small_ref, variant):
    c, J_ref, g_ref = small_ref
    say(f"[gpu] adjoint {c['shape']} porous, {c['steps']} steps, variant {variant}")
    g, lat = gpu_gradient(c, every=7, variant=variant)
    assert lat.info["variant"] == variant
    m = c["flags"] == 0
    err = rel_l2(g, g_ref, m)
    J = float(lbm.outlet_flux(lat))
    say(f"  rel-L2(dJ/dF_x) = {err:.3e}; J = {J:.6e} (oracle {J_ref:.6e})")
    assert err <= TOL_GRAD
    assert abs(J - J_ref) <= 1e-5 * abs(J_ref)
    assert np.all(g[~m] == 0.0)
    lat.close()


@pytest.mark.parametrize("every", [1, 4, 7, 50])
def test_checkpoint_interval_does_not_change_the_gradient(every):
    """Recomputed stretches give the moments the forward pass gave: the same
    gradient bits for one stretch (every = 30 or more), stretches of one
    step (each recomputed step writes its moments only), and a shorter last
    stretch."""
    c = small_case(steps=30)
    g1, l1 = gpu_gradient(c, every=30)
    g2, l2 = gpu_gradient(c, every=every)
    assert np.array_equal(g1, g2)
    l1.close()
    l2.close()


def test_outlet_flux_with_a_partial_last_workgroup_of_rows():
    """lb_outlet_flux sums in two passes (one row per lane, a part per
    workgroup, then the parts in order). ny * nz = 1200 rows leave a partial
    last workgroup; the value equals the oracle's flux of the same stored
    state up to FP64 rounding."""
    c = small_case(nx=24, ny=40, nz=30, steps=10, seed=5)
    lat = gpu_lattice(c)
    lat.step(c["steps"])
    J = float(lbm.outlet_flux(lat))
    S = lat.get_f().astype(np.float64) + W19.reshape(19, 1, 1, 1)
    # the library holds the uniform force in FP32 (the kernels' arithmetic)
    F32 = tuple(float(np.float32(f)) for f in c["force"])
    J_ref = oracle.outlet_flux(S, F=F32, flags=c["flags"], Fx_field=c["fx"].astype(np.float64))
    say(f"  outlet flux 24x40x30: {J:.12e} (oracle of the same state {J_ref:.12e})")
    assert abs(J - J_ref) <= 1e-12 * max(1.0, abs(J_ref))
    lat.close()


def test_lattice_ends_where_lb_step_ends():
    """The gradient call advances the lattice exactly as lb_step does."""
    torch = require_gpu()
    c = small_case(steps=40)
    _, lat1 = gpu_gradient(c, every=9)
    lat2 = gpu_lattice(c)
    lat2.step(c["steps"])
    assert lat1.steps_done == lat2.steps_done == c["steps"]
    assert np.array_equal(lat1.get_f(), lat2.get_f())
    assert np.array_equal(lat1.sums(c["steps"]), lat2.sums(c["steps"]))
    lat1.close()
    lat2.close()


def test_gradient_matches_gpu_finite_differences():
    """Central differences of the GPU's FP32 forward model at a few cells
    (J is nearly linear in the force, so a step of 2e-5 keeps truncation
    small while the difference stays far above FP32 noise)."""
    torch = require_gpu()
    c = small_case(steps=50)
    g, lat = gpu_gradient(c, every=10)
    lat.close()
    rng = np.random.default_rng(23)
    fluid = np.argwhere(c["flags"] == 0)
    cells = [tuple(fluid[k]) for k in rng.choice(len(fluid), 5, replace=False)]
    h = 2e-5
    for cell in cells:
        Js = []
        for sgn in (1, -1):
            cc = dict(c)
            fx = c["fx"].copy()
            fx[cell] += sgn * h
            cc["fx"] = fx
            lt = gpu_lattice(cc)
            lt.step(c["steps"])
            Js.append(float(lbm.outlet_flux(lt)))
            lt.close()
        fd = (Js[0] - Js[1]) / (2 * h)
        say(f"  cell {cell}: adjoint {g[cell]:.6e}, finite difference {fd:.6e}")
        assert abs(fd - g[cell]) <= 2e-3 * max(abs(fd), 1e-2)


def test_autograd_function(small_ref):
    torch = require_gpu()
    c, J_ref, g_ref = small_ref
    lat = gpu_lattice(c)
    fx = torch.from_numpy(c["fx"]).cuda().requires_grad_(True)
    J = lbm.outlet_flux_autograd(fx, lat, c["steps"], 7)
    J.backward()
    Jv = J.detach().item()
    g = fx.grad.double().cpu().numpy()
    m = c["flags"] == 0
    err = rel_l2(g, g_ref, m)
    say(f"  autograd: J = {Jv:.6e}, rel-L2(grad) = {err:.3e}")
    assert abs(Jv - J_ref) <= 1e-5 * abs(J_ref)
    assert err <= TOL_GRAD
    lat.close()


GOLDEN = os.path.join(HERE, "golden", "porous128_grad500.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored oracle gradient missing")
def test_porous128_500_steps_vs_stored_oracle_gradient():
    """128^3 porous channel (porosity 0.85), force 1e-6, 500 steps,
    checkpoints every 50: J and dJ/dF_x against the stored FP64 oracle."""
    torch = require_gpu()
    gold = json.load(open(GOLDEN))
    cfg = inputs.porous_channel(128, porosity=0.85, tau=0.6, g=1e-6, seed=4, steps=500, every=50)
    n = 128
    say(f"[gpu] adjoint porous 128^3, {cfg['steps']} steps, checkpoints every {cfg['every']}")
    lat = lbm.Lattice(n, n, n, cfg["tau"], flags=cfg["flags"])
    lat.set_force(*cfg["force"])
    lat.init_eq(torch.from_numpy(cfg["rho"]).cuda(), torch.from_numpy(cfg["u"]).cuda())
    lat.set_force_field(torch.zeros((n, n, n), dtype=torch.float32, device="cuda"))
    J, g = lat.grad_outlet_flux_x(cfg["steps"], cfg["every"])
    g = g.double()
    idx = torch.tensor(gold["cells_zyx"], device="cuda")
    gs = g[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    ref = np.array(gold["grad"])
    err = float(np.linalg.norm(gs - ref) / np.linalg.norm(ref))
    l2 = float(torch.linalg.norm(g))
    say(f"  J = {J:.8e} (oracle {gold['J']:.8e}); sampled rel-L2(grad) = {err:.3e}; "
        f"|grad| = {l2:.6e} (oracle {gold['grad_l2']:.6e})")
    assert abs(J - gold["J"]) <= 1e-5 * abs(gold["J"])
    assert err <= TOL_GRAD
    assert abs(l2 - gold["grad_l2"]) <= TOL_GRAD * gold["grad_l2"]
    lat.close()

"""In-place (one-array, "AA" pattern) storage against two-array storage
(needs an MI355X).

Both run the same per-site arithmetic on the same values, so after any
number of steps the state, the macroscopic fields and the FP64 totals must
be identical bit for bit; two-array storage is itself checked against the
FP64 oracle in test_parity.py.  The odd-phase array holds the state pulled
to the next step's sites, so reading it back exercises the reconstruction.
"""
import numpy as np
import pytest

import oracle
import paper_2409_16781_amd as lbm
from paper_2409_16781_amd import inputs
from gpu_util import require_gpu, say, streamed_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    require_gpu()
    oracle.build(force=False)


def case(kind, nx=32, ny=16, nz=8, seed=5):
    rng = np.random.default_rng(seed)
    iz, iy, ix = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    rho, u = inputs.smooth_fields(np, iz, iy, ix, max(nx, ny, nz), amp=0.02)
    rho = np.ascontiguousarray(rho + rng.uniform(-1e-4, 1e-4, rho.shape))
    flags, F = None, (0.0, 0.0, 0.0)
    if kind == "walls":
        flags, F = inputs.channel_flags(nx, ny, nz), (1e-5, 0.0, 2e-6)
    elif kind == "porous":
        flags, F = inputs.random_flags(nx, ny, nz, 0.15, seed + 1), (1e-5, -2e-6, 0.0)
    return dict(shape=(nz, ny, nx), rho=rho, u=np.ascontiguousarray(u), flags=flags, tau=0.7, force=F)


def make(c, codec, inplace):
    torch = require_gpu()
    nz, ny, nx = c["shape"]
    lat = lbm.Lattice(nx, ny, nz, c["tau"], flags=c["flags"], codec=codec, inplace=inplace)
    lat.set_force(*c["force"])
    lat.init_eq(torch.from_numpy(c["rho"]).cuda(), torch.from_numpy(c["u"]).cuda())
    return lat


def fluid(c):
    return np.ones(c["shape"], bool) if c["flags"] is None else c["flags"] == 0


@pytest.mark.parametrize("steps", [1, 2, 5, 70])
@pytest.mark.parametrize("kind", ["fluid", "walls", "porous"])
@pytest.mark.parametrize("codec", ["f32", "f16", "bf16"])
def test_inplace_equals_two_arrays(codec, kind, steps):
    c = case(kind)
    a = make(c, codec, False)
    b = make(c, codec, True)
    assert b.info["inplace"] == 1 and a.info["inplace"] == 0
    say(f"[gpu] in-place vs two arrays: {kind} {c['shape']} {codec}, {steps} steps, variant {b.info['variant']}")
    a.step(steps)
    b.step(steps)
    m = fluid(c)
    fa, fb = a.get_f(), b.get_f()
    assert np.array_equal(fa[:, m], fb[:, m])
    ra, ua = a.macros()
    rb, ub = b.macros()
    assert np.array_equal(ra.cpu().numpy(), rb.cpu().numpy())
    assert np.array_equal(ua.cpu().numpy(), ub.cpu().numpy())
    assert np.array_equal(a.sums(steps), b.sums(steps))
    a.close()
    b.close()


@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_inplace_step_macros(codec):
    """With in-place storage lb_step_macros derives the fields from the state
    just written (a second kernel): equal to the in-pass moments of two-array
    storage up to the rounding of the stored values (an FP16 unit in the last
    place of f - w ~ 1e-2 is 7.6e-6; FP32: 1e-9)."""
    c = case("walls")
    a = make(c, codec, False)
    b = make(c, codec, True)
    ra, ua = a.step_macros(7)
    rb, ub = b.step_macros(7)
    m = fluid(c)
    tol_r, tol_u = (2e-7, 1e-8) if codec == "f32" else (5e-5, 5e-6)
    assert np.abs(ra.cpu().numpy() - rb.cpu().numpy())[m].max() < tol_r
    assert np.abs(ua.cpu().numpy() - ub.cpu().numpy()).max() < tol_u
    assert np.array_equal(a.get_f()[:, m], b.get_f()[:, m])
    a.close()
    b.close()


def test_inplace_checkpoint_resume_at_odd_phase():
    c = case("porous")
    b1 = make(c, "f32", True)
    b1.step(3)                      # odd phase
    ckpt = b1.get_f()
    b1.step(4)
    b2 = make(c, "f32", True)
    b2.set_f(ckpt)
    b2.step(4)
    m = fluid(c)
    assert np.array_equal(b1.get_f()[:, m], b2.get_f()[:, m])
    b1.close()
    b2.close()


def test_inplace_pure_streaming_matches_oracle():
    """omega = 0: three in-place steps permute the values exactly as the oracle does."""
    import math

    c = case("porous")
    nz, ny, nx = c["shape"]
    lat = lbm.Lattice(nx, ny, nz, math.inf, flags=c["flags"], inplace=True)
    rng = np.random.default_rng(9)
    raw = rng.uniform(-0.01, 0.01, (19, nz, ny, nx)).astype(np.float32)
    lat.set_f(raw)
    lat.step(3)
    out, ref = streamed_pair(lat.get_f().astype(np.float64), raw.astype(np.float64), 3, c["flags"])
    m = fluid(c)
    assert np.array_equal(out[:, m], ref[:, m])
    lat.close()


def test_inplace_rejects_rows_that_do_not_tile():
    with pytest.raises(lbm.LBError, match="in-place"):
        lbm.Lattice(96, 8, 8, 0.7, inplace=True)


@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_inplace_512_cube_equals_two_arrays(codec):
    torch = require_gpu()
    n, steps = 512, 9
    cfg = inputs.tgv_noise_box(n, u0=0.01, tau=0.55, steps=steps, noise=1e-3, seed=2)
    say(f"[gpu] in-place 512^3 {codec}, {steps} steps")
    rho = torch.from_numpy(cfg["rho"]).cuda()
    u = torch.from_numpy(cfg["u"]).cuda()
    outs = []
    for inplace in (False, True):
        lat = lbm.Lattice(n, n, n, cfg["tau"], codec=codec, inplace=inplace)
        lat.init_eq(rho, u)
        lat.step(steps)
        r, uu = lat.macros()
        outs.append((uu, lat.sums(steps)))
        del r
        lat.close()
        torch.cuda.empty_cache()
    assert torch.equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])

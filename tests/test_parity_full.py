"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

* 512^3 Taylor-Green vortex, 1000 steps: a state uniform in z evolves exactly
  as the nz = 1 lattice (every site does the same arithmetic; the oracle
  checks this bit for bit), so the whole 512^3 field is compared with an FP64
  oracle run on 512 x 512 x 1 sites.
* 512^3 Taylor-Green vortex with seeded U(+-1e-3) velocity noise (the timed
  workload): sampled sites after 16 steps against the light-cone oracle (a
  site after n steps depends only on the initial state within distance n),
  and after 200 and 1000 steps against stored FP64 oracle results of the
  whole run (16384 seeded sites, plus whole-field mode amplitude, energy and
  mass), for FP32, FP16, scaled 16-bit and BF16 storage.
* 256 x 128 x 128 channel, 5000 steps: sampled sites, the x-z averaged
  profile and the conservation totals against stored FP64 oracle results
  (tests/golden/channel256x128x128_5000.json, written by
  tests/golden/make_channel_golden.py from the oracle alone).
* Largest lattices: 1280^3 (2.1e9 sites, near the 2^31-site index limit) with
  FP16 storage and 1024^3 with FP32 storage, sampled sites after 4 steps.

Bounds: relative L2 error of u <= 1e-5 (FP32 storage) and <= 2e-3 (FP16 and
scaled 16-bit); BF16 storage is held to the same 2e-3 bound and fails it (an
expected failure, with the measured error).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import paper_2409_16781_amd as lbm
from paper_2409_16781_amd import inputs
from gpu_util import bf16_bound, require_gpu, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"f32": 1e-5, "f16": 2e-3, "bf16": 2e-3, "s16": 2e-3}


@pytest.fixture(scope="module", autouse=True)
def _setup():
    require_gpu()
    oracle.build(force=False)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ----------------------------------------------- 512^3 TGV, 1000 steps -----

@pytest.fixture(scope="module")
def tgv512_ref():
    n, tau, steps = 512, 0.55, 1000
    r2, u2 = inputs.tgv_fields(n, n, 1, 0.01)
    S = oracle.run(oracle.init((1, n, n), r2, u2), tau, steps)
    _, u_ref = oracle.macros(S)
    return dict(n=n, tau=tau, steps=steps, r2=r2, u2=u2, u_ref=u_ref[:, 0])


@pytest.mark.parametrize("codec", ["f32", "f16", "bf16"])
def test_tgv512_1000_steps_whole_field(tgv512_ref, codec):
    torch = require_gpu()
    c = tgv512_ref
    n = c["n"]
    say(f"[gpu] tgv512 z-uniform {codec} {c['steps']} steps")
    lat = lbm.Lattice(n, n, n, c["tau"], codec=codec)
    rho = torch.from_numpy(c["r2"]).cuda().expand(n, n, n).contiguous()
    u = torch.from_numpy(c["u2"]).cuda().expand(3, n, n, n).contiguous()
    lat.init_eq(rho, u)
    del rho, u
    lat.step(c["steps"])
    sums = lat.sums(c["steps"])
    r_g, u_g = lat.macros()
    # every z plane is the same computation: bit-identical planes
    assert torch.equal(u_g, u_g[:, :1].expand(3, n, n, n))
    err = rel_l2(u_g[:, 0].double().cpu().numpy(), c["u_ref"])
    drift = abs(sums[-1, 0] - sums[0, 0]) / sums[0, 0]
    say(f"  rel-L2(u) = {err:.3e} over all {n}^3 sites; mass drift over {c['steps']} steps {drift:.2e}")
    if codec == "bf16":
        bf16_bound(err)
    assert err <= TOL[codec]
    lat.close()
    torch.cuda.empty_cache()


# ----------------------------------------- 512^3 TGV + noise, light cone -----

@pytest.fixture(scope="module")
def tgv512_noise():
    return inputs.tgv_noise_box(512, u0=0.01, tau=0.55, steps=1000, noise=1e-3, seed=2)


@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_tgv512_noise_sampled_sites(tgv512_noise, codec):
    torch = require_gpu()
    cfg = tgv512_noise
    n, steps = 512, 16
    say(f"[gpu] tgv512 + noise {codec}, {steps} steps, light-cone samples")
    lat = lbm.Lattice(n, n, n, cfg["tau"], codec=codec)
    lat.init_eq(torch.from_numpy(cfg["rho"]).cuda(), torch.from_numpy(cfg["u"]).cuda())
    torch.cuda.empty_cache()
    lat.step(steps)
    r_g, u_g = lat.macros()
    rng = np.random.default_rng(5)
    centres = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(24)]
    centres += [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 0), (n - 1, 0, n - 1)]
    idx = torch.tensor(centres, device="cuda")
    ug = u_g[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.double().cpu().numpy()
    rr, ur = oracle.run_window(cfg["rho"], cfg["u"], None, cfg["tau"], steps, centres)
    err = rel_l2(ug, ur)
    say(f"  rel-L2(u) over {len(centres)} sampled sites = {err:.3e}")
    assert err <= TOL[codec]
    lat.close()
    torch.cuda.empty_cache()


# ------------------------ 512^3 TGV + noise, 1000 steps, stored oracle -----
# tests/golden/tgv512_noise_golden.{json,npz}: the FP64 oracle's u and rho at
# 16384 seeded sites and whole-field statistics after 200 and 1000 steps of
# this exact workload, written by make_tgv512_noise_golden.py from the oracle
# alone.

NOISE_GOLDEN = os.path.join(HERE, "golden", "tgv512_noise_golden")


@pytest.fixture(scope="module")
def noise_golden():
    with open(NOISE_GOLDEN + ".json") as f:
        meta = json.load(f)
    with np.load(NOISE_GOLDEN + ".npz") as z:
        arr = {k: z[k] for k in z.files}
    return meta, arr


def field_stats_gpu(torch, rho, u):
    """The generator's whole-field statistics, evaluated on the GPU result in FP64."""
    n = rho.shape[-1]
    k = 2.0 * math.pi / n
    x = torch.arange(n, dtype=torch.float64, device=rho.device)
    mx = torch.outer(torch.cos(k * x), torch.sin(k * x))    # (y, x): sin kx cos ky
    my = -torch.outer(torch.sin(k * x), torch.cos(k * x))   # -cos kx sin ky
    ux, uy = u[0].double(), u[1].double()
    proj = float((ux * mx).sum() + (uy * my).sum())
    norm = float(rho.shape[0] * ((mx * mx).sum() + (my * my).sum()))
    return dict(mode_amplitude=proj / norm,
                sum_u2=[float((u[a].double() ** 2).sum()) for a in range(3)])


@pytest.mark.skipif(not os.path.exists(NOISE_GOLDEN + ".npz"), reason="stored 512^3 oracle results missing")
@pytest.mark.parametrize("codec", ["f32", "f16", "s16", "bf16"])
def test_tgv512_noise_1000_steps_vs_stored_oracle(tgv512_noise, noise_golden, codec):
    """The timed workload itself, at its stated 1000 steps: u at 16384 seeded
    sites against the FP64 oracle (rel-L2 <= 1e-5 FP32, <= 2e-3 16-bit), the
    amplitude of the Taylor-Green mode and the energy per component over the
    whole field, and the mass total."""
    torch = require_gpu()
    meta, arr = noise_golden
    cfg = tgv512_noise
    n = 512
    say(f"[gpu] tgv512 + noise {codec}: 1000 steps against the stored oracle results")
    lat = lbm.Lattice(n, n, n, cfg["tau"], codec=codec)
    lat.init_eq(torch.from_numpy(cfg["rho"]).cuda(), torch.from_numpy(cfg["u"]).cuda())
    torch.cuda.empty_cache()
    idx = torch.from_numpy(arr["sites_zyx"]).cuda()
    done, err = 0, None
    for k in (200, 1000):
        lat.step(k - done)
        done = k
        r_g, u_g = lat.macros()
        ug = u_g[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.double().cpu().numpy()
        err = rel_l2(ug, arr[f"u_{k}"])
        st = field_stats_gpu(torch, r_g, u_g)
        ref = meta["checkpoints"][str(k)]
        mode_err = abs(st["mode_amplitude"] - ref["mode_amplitude"]) / abs(ref["mode_amplitude"])
        e2_err = max(abs(st["sum_u2"][a] - ref["sum_u2"][a]) / ref["sum_u2"][a] for a in (0, 1))
        mass = lat.sums(1)[0, 0]
        mass_err = abs(mass - ref["sums"][0]) / ref["sums"][0]
        say(f"  {k} steps: rel-L2(u) at {len(idx)} sites = {err:.3e}; mode amplitude {mode_err:.2e}, "
            f"energy {e2_err:.2e}, mass {mass_err:.2e} (relative differences)")
        del r_g, u_g
        if codec != "bf16":  # BF16: reported, an expected failure of the bound
            assert err <= TOL[codec]
            assert mode_err <= TOL[codec] and e2_err <= 2 * TOL[codec]
            assert mass_err <= 1e-8
    lat.close()
    torch.cuda.empty_cache()
    if codec == "bf16":
        bf16_bound(err)


# --------------------------------------------- channel, 5000 steps ---------

GOLDEN = os.path.join(HERE, "golden", "channel256x128x128_5000.json")


def _channel_5000(codec):
    torch = require_gpu()
    gold = json.load(open(GOLDEN))
    cfg = inputs.channel(256, 128, 128, tau=0.6, g=1e-6, steps=5000, noise=1e-4, seed=1)
    nz, ny, nx = cfg["shape"]
    say(f"[gpu] channel 256x128x128 {codec} 5000 steps")
    lat = lbm.Lattice(nx, ny, nz, cfg["tau"], flags=cfg["flags"], codec=codec)
    lat.set_force(*cfg["force"])
    lat.init_eq(torch.from_numpy(cfg["rho"]).cuda(), torch.from_numpy(cfg["u"]).cuda())
    lat.step(gold["steps"])
    sums = lat.sums(1)[0]
    r_g, u_g = lat.macros()
    idx = torch.tensor(gold["sites_zyx"], device="cuda")
    ug = u_g[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.double().cpu().numpy()
    err = rel_l2(ug, np.array(gold["u"]))
    prof = u_g[0].double().mean(dim=(0, 2)).cpu().numpy()
    perr = rel_l2(prof[1:-1], np.array(gold["profile_ux"])[1:-1])
    dmass = abs(sums[0] - gold["sums"][0]) / gold["sums"][0]
    say(f"  rel-L2(u) sampled = {err:.3e}, profile = {perr:.3e}; relative mass difference {dmass:.2e}")
    lat.close()
    torch.cuda.empty_cache()
    return err, perr, dmass


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored channel results missing")
def test_channel_5000_steps_vs_stored_oracle():
    """The channel workload is specified with FP32 storage."""
    err, perr, dmass = _channel_5000("f32")
    assert err <= TOL["f32"]
    assert perr <= TOL["f32"]
    assert dmass < 1e-10


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="stored channel results missing")
def test_channel_5000_steps_fp16_storage_reported():
    """FP16 storage on the channel, measured and reported (not a target).

    Each step the force changes a population by about 3 (1 - omega/2) w F
    ~ 3e-8, below half an FP16 unit in the last place of f - w near the
    channel centre (~5e-7), so round-to-nearest storage keeps part of the
    increments from accumulating; the error is of order 1e-2 here.  The
    sanity bound only guards against a broken kernel."""
    err, perr, dmass = _channel_5000("f16")
    assert np.isfinite(err) and err < 5e-2


def test_channel_full_size_light_cone():
    """The 256x128x128 channel with walls and force, sampled after 40 steps
    against the light-cone oracle (independent of the stored results)."""
    torch = require_gpu()
    cfg = inputs.channel(256, 128, 128, tau=0.6, g=1e-6, steps=40, noise=1e-4, seed=1)
    nz, ny, nx = cfg["shape"]
    steps = 40
    lat = lbm.Lattice(nx, ny, nz, cfg["tau"], flags=cfg["flags"], codec="f32")
    lat.set_force(*cfg["force"])
    lat.init_eq(torch.from_numpy(cfg["rho"]).cuda(), torch.from_numpy(cfg["u"]).cuda())
    lat.step(steps)
    _, u_g = lat.macros()
    rng = np.random.default_rng(6)
    centres = [(int(rng.integers(0, nz)), int(rng.integers(1, ny - 1)), int(rng.integers(0, nx))) for _ in range(6)]
    centres += [(0, 1, 0), (nz - 1, ny - 2, nx - 1)]
    idx = torch.tensor(centres, device="cuda")
    ug = u_g[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.double().cpu().numpy()
    _, ur = oracle.run_window(cfg["rho"], cfg["u"], cfg["flags"], cfg["tau"], steps, centres, F=cfg["force"])
    err = rel_l2(ug, ur)
    say(f"  channel light-cone rel-L2(u) = {err:.3e}")
    assert err <= 1e-5
    lat.close()


# ------------------------------------------------- largest lattices --------

@pytest.mark.parametrize("codec,n", [("f16", 1280), ("f32", 1024)])
def test_largest_lattice_sampled_sites(codec, n):
    torch = require_gpu()
    steps = 4
    say(f"[gpu] {n}^3 {codec} ({n ** 3 / 1e9:.2f}e9 sites), {steps} steps")
    lat = lbm.Lattice(n, n, n, 0.7, codec=codec)
    lat.set_force(2e-5, -1e-5, 5e-6)
    ar = torch.arange(n, device="cuda", dtype=torch.float64)
    # analytic initial fields evaluated on the device plane by plane
    u = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
    rho = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
    for z in range(n):
        r_z, u_z = inputs.smooth_fields(torch, torch.tensor(float(z), device="cuda", dtype=torch.float64),
                                        ar[:, None], ar[None, :], n)
        rho[z] = r_z
        u[:, z] = u_z
    lat.init_eq(rho, u)
    del rho, u
    torch.cuda.empty_cache()
    lat.step(steps)
    sums = lat.sums(steps)
    assert np.all(np.isfinite(sums))
    r_g, u_g = lat.macros()
    centres = [(0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, 3, n - 2), (7, n // 3, 11), (n - 3, n // 2, n // 2)]
    idx = torch.tensor(centres, device="cuda")
    ug = u_g[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.double().cpu().numpy()
    _, ur = oracle.run_window(None, None, None, 0.7, steps, centres, F=(2e-5, -1e-5, 5e-6), shape=(n, n, n),
                              fields=lambda iz, iy, ix: inputs.smooth_fields(np, iz, iy, ix, n))
    err = rel_l2(ug, ur)
    say(f"  rel-L2(u) sampled = {err:.3e}")
    assert err <= TOL[codec]
    lat.close()
    del r_g, u_g
    torch.cuda.empty_cache()

"""GPU parity of lattice batches (many domains, one launch per step) against
the FP64 oracle, domain by domain (needs an MI355X).

Domains of a batch never interact, so every domain of a batch run must match
the oracle run of that domain alone: rel-L2(u) <= 1e-5 with FP32 storage and
<= 2e-3 with FP16 storage, bit-exact where the method is a permutation
(omega = 0) or a fixed point (rest).  The shapes cover rows that are padded
to whole vectors (nx not a multiple of the vector width), rows whose tiles
exchange x-edges through LDS, a 1x1x1 domain, walls, porous media, per-domain
relaxation times and forces, every kernel variant, and the 64-domain porous
workload at its full size and step count.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2409_16781_amd as lbm
from paper_2409_16781_amd import inputs
from gpu_util import (FP64_SUM_TOL, decode_raw, exact_state_totals, fluid_mask, oracle_run, rel_l2_u, require_gpu, say,
                      streamed_pair, totals_gap_bound)

pytestmark = pytest.mark.gpu

TOL_U = {"f32": 1e-5, "f16": 2e-3}


@pytest.fixture(scope="module", autouse=True)
def _setup():
    require_gpu()
    oracle.build(force=False)


def mixed_domains():
    """Six small domains with different shapes, geometry, tau and force."""
    doms = []
    specs = [
        # (nx, ny, nz), tau, flags kind, force
        ((32, 16, 8), 0.6, "random", (2e-5, 0.0, -1e-5)),
        ((17, 9, 11), 0.9, "spheres", (1e-5, 0.0, 0.0)),
        ((5, 7, 6), 0.55, None, (0.0, 3e-5, 0.0)),
        ((1, 1, 1), 0.7, None, (1e-5, 2e-5, -3e-5)),
        ((23, 12, 10), 0.75, "walls", (1e-5, 0.0, 0.0)),
        ((64, 6, 5), 1.0, None, (0.0, 0.0, 0.0)),
    ]
    for k, ((nx, ny, nz), tau, kind, F) in enumerate(specs):
        if kind == "random":
            flags = inputs.random_flags(nx, ny, nz, 0.1, 100 + k)
        elif kind == "spheres":
            flags = inputs.sphere_flags(nx, ny, nz, 0.8, 200 + k)
        elif kind == "walls":
            flags = inputs.channel_flags(nx, ny, nz)
        else:
            flags = None
        iz, iy, ix = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                                 np.arange(nx, dtype=np.float64), indexing="ij")
        rho, u = inputs.smooth_fields(np, iz, iy, ix, max(nx, ny, nz), amp=0.02)
        rho = rho + inputs.uniform_noise((nz, ny, nx), 1e-4, 300 + k)
        doms.append(dict(name=f"mixed{k}", shape=(nz, ny, nx), rho=np.ascontiguousarray(rho),
                         u=np.ascontiguousarray(u), flags=flags, tau=tau, force=F))
    return doms


def make_batch(doms, codec="f32", variant=None, autotune=False, init=True):
    torch = require_gpu()
    import os

    old = os.environ.get("LB_BATCH_KERNEL")
    if variant is not None:
        os.environ["LB_BATCH_KERNEL"] = str(variant)
    try:
        b = lbm.Batch([(d["shape"][2], d["shape"][1], d["shape"][0]) for d in doms], [d["tau"] for d in doms],
                      flags=[d["flags"] for d in doms], codec=codec, autotune=autotune)
    finally:
        if old is None:
            os.environ.pop("LB_BATCH_KERNEL", None)
        else:
            os.environ["LB_BATCH_KERNEL"] = old
    for k, d in enumerate(doms):
        b.set_force(*d["force"], domain=k)
        if init:
            rho = torch.from_numpy(np.ascontiguousarray(d["rho"], np.float64)).cuda()
            u = torch.from_numpy(np.ascontiguousarray(d["u"], np.float64)).cuda()
            b.init_eq(k, rho, u)
    return b


@pytest.fixture(scope="module")
def mixed_ref():
    doms = mixed_domains()
    steps = 60
    refs = [oracle_run(d, steps) for d in doms]
    return doms, steps, refs


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_mixed_batch_matches_oracle_per_domain(mixed_ref, codec, variant):
    doms, steps, refs = mixed_ref
    say(f"[gpu] batch of {len(doms)} mixed domains, {codec}, variant {variant}, {steps} steps")
    b = make_batch(doms, codec, variant)
    assert b.info["variant"] == variant
    b.step(steps)
    for k, (d, (r_ref, u_ref, _)) in enumerate(zip(doms, refs)):
        r, u = b.macros(k)
        u = u.double().cpu().numpy()
        m = fluid_mask(d)
        err = rel_l2_u(u, u_ref, m)
        say(f"  domain {k} {d['shape']} tau={d['tau']}: rel-L2(u) = {err:.3e}")
        assert err <= TOL_U[codec]
        r = r.double().cpu().numpy()
        assert np.all(r[~m] == 0.0)
        assert np.abs(r[m] - r_ref[m]).max() < (1e-6 if codec == "f32" else 1e-4)
    b.close()


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_pure_streaming_is_exact_per_domain(codec, variant, walls):
    """omega = 0, F = 0: three steps permute each domain's values exactly as
    the oracle permutes them."""
    shapes = [(9, 5, 7), (32, 8, 4), (6, 3, 5), (1, 1, 1)]
    rng = np.random.default_rng(71)
    doms = []
    for k, (nx, ny, nz) in enumerate(shapes):
        flags = inputs.random_flags(nx, ny, nz, 0.2, 80 + k) if walls else None
        doms.append(dict(shape=(nz, ny, nx), tau=math.inf, flags=flags, force=(0.0, 0.0, 0.0)))
    b = make_batch(doms, codec, variant, init=False)
    raws = []
    for k, d in enumerate(doms):
        g = rng.uniform(-0.01, 0.01, (19,) + d["shape"])
        raw = g.astype(np.float32) if codec == "f32" else g.astype(np.float16).view(np.uint16)
        raws.append(raw)
        b.set_f(k, raw)
    b.step(3)
    for k, d in enumerate(doms):
        out, ref = streamed_pair(lbm.decode_state(b.get_f(k), codec), lbm.decode_state(raws[k], codec), 3, d["flags"])
        m = fluid_mask(d)
        assert np.array_equal(out[:, m], ref[:, m]), f"domain {k}"
    b.close()


def test_rest_state_is_exactly_invariant():
    doms = [dict(shape=(8, 12, 16), tau=0.7, flags=inputs.channel_flags(16, 12, 8), force=(0.0, 0.0, 0.0)),
            dict(shape=(3, 5, 7), tau=0.9, flags=None, force=(0.0, 0.0, 0.0))]
    for codec in ("f32", "f16", "bf16"):
        b = make_batch(doms, codec, init=False)
        b.step(70)
        for k in range(len(doms)):
            assert not np.any(b.get_f(k))
        b.close()


def test_totals_per_domain_match_oracle(mixed_ref):
    doms, steps, refs = mixed_ref
    b = make_batch(doms, "f32")
    b.step(steps)
    for k, (d, (_, _, S)) in enumerate(zip(doms, refs)):
        tot = b.sums(k, 1)[0]
        ref = oracle.sums(S, d["flags"])
        g = decode_raw(b.get_f(k), "f32")
        m = fluid_mask(d)
        bound = totals_gap_bound(g, S, m)
        say(f"  domain {k}: totals - oracle totals = {tot - ref}, bound {bound}")
        # the totals are the FP64 sums of the stored state itself ...
        exact, scale = exact_state_totals(g, m)
        assert np.all(np.abs(tot - exact) <= FP64_SUM_TOL * scale), (k, tot, exact, scale)
        # ... so they differ from the FP64 oracle's by the summed difference of
        # the FP32 state from the oracle's state only
        assert np.all(np.abs(tot - ref) <= bound), (k, tot - ref, bound)
    b.close()


def test_graph_replay_equals_eager_steps():
    doms = mixed_domains()
    b1 = make_batch(doms, "f32")
    b1.step(70)  # 70 >= 64: one captured graph of the whole run
    b1.step(65)  # odd runs: captured from each parity
    b1.step(65)
    total = 200
    b2 = make_batch(doms, "f32")
    for _ in range(total):
        b2.step(1)
    for k in range(len(doms)):
        assert np.array_equal(b1.get_f(k), b2.get_f(k)), k
        # every domain's whole ring of per-step totals, chained runs vs single steps
        assert np.array_equal(b1.sums(k, total), b2.sums(k, total)), k
    b1.close()
    b2.close()


@pytest.mark.parametrize("codec", ["f32", "f16"])
def test_checkpoint_resume_is_exact(codec):
    doms = mixed_domains()
    b1 = make_batch(doms, codec)
    b1.step(10)
    ckpt = [b1.get_f(k) for k in range(len(doms))]
    b1.step(15)
    b2 = make_batch(doms, codec, init=False)
    for k, c in enumerate(ckpt):
        b2.set_f(k, c)
    b2.step(15)
    for k in range(len(doms)):
        assert np.array_equal(b1.get_f(k), b2.get_f(k)), k
    b1.close()
    b2.close()


def test_autotuned_shape_matches_default():
    doms = mixed_domains()
    b1 = make_batch(doms, "f32")
    b2 = make_batch(doms, "f32", autotune=True)
    say(f"  autotuned shape: {b2.info}")
    assert b2.info["autotuned"] == 1
    b1.step(40)
    b2.step(40)
    for k, d in enumerate(doms):
        _, u1 = b1.macros(k)
        _, u2 = b2.macros(k)
        u1, u2 = u1.double().cpu().numpy(), u2.double().cpu().numpy()
        m = fluid_mask(d)
        if np.any(u1[:, m]):
            assert rel_l2_u(u2, u1, m) <= 1e-6, k
    b1.close()
    b2.close()


@pytest.mark.parametrize("cap", [4, 5])
def test_workgroup_cap_changes_nothing_but_occupancy(cap, monkeypatch):
    """A cap on the resident workgroups per CU (dynamic LDS on the 4-byte
    kernel, one of the autotuner's candidates) gives the same state and the
    same totals, bit for bit."""
    doms = mixed_domains()
    monkeypatch.setenv("LB_BATCH_KERNEL", "3")
    b1 = make_batch(doms, "f32")
    monkeypatch.setenv("LB_BATCH_WG_CAP", str(cap))
    b2 = make_batch(doms, "f32")
    assert b1.info["wg_cap"] == 0 and b2.info["wg_cap"] == cap
    say(f"  4-byte batch kernel, cap {cap} workgroups per CU")
    b1.step(70)
    b2.step(70)
    for k in range(len(doms)):
        assert np.array_equal(b1.get_f(k), b2.get_f(k)), k
        assert np.array_equal(b1.sums(k, 70), b2.sums(k, 70)), k
    b1.close()
    b2.close()


def test_invalid_workgroup_cap_is_refused(monkeypatch):
    monkeypatch.setenv("LB_BATCH_WG_CAP", "2")
    with pytest.raises(lbm.LBError):
        make_batch(mixed_domains()[:1], "f32")


def test_batch_domain_equals_single_lattice():
    """A domain advanced inside a batch matches the same lattice advanced
    alone through lb_step (same arithmetic per site)."""
    torch = require_gpu()
    doms = mixed_domains()
    b = make_batch(doms, "f32")
    b.step(30)
    for k in (0, 1, 4):
        d = doms[k]
        nz, ny, nx = d["shape"]
        lat = lbm.Lattice(nx, ny, nz, d["tau"], flags=d["flags"])
        lat.set_force(*d["force"])
        lat.init_eq(torch.from_numpy(d["rho"]).cuda(), torch.from_numpy(d["u"]).cuda())
        lat.step(30)
        _, u1 = lat.macros()
        _, u2 = b.macros(k)
        m = fluid_mask(d)
        err = rel_l2_u(u2.double().cpu().numpy(), u1.double().cpu().numpy(), m)
        say(f"  domain {k}: batch vs single lattice rel-L2(u) = {err:.2e}")
        assert err <= 1e-6
        lat.close()
    b.close()


def test_batch64_full_workload_sampled_domains():
    """The 64-domain porous workload (extents U{16..96}, porosity 0.8, tau
    U[0.55, 1.0], force 1e-6, 500 steps) in one launch per step, in the
    autotuned shape; four domains checked against the oracle run alone."""
    doms = inputs.batch_domains(64, seed=3)
    steps = 500
    say(f"[gpu] batch64 porous, {steps} steps, {sum(int(np.prod(d['shape'])) for d in doms)} sites")
    b = make_batch(doms, "f32", autotune=True)
    say(f"  shape: {b.info}")
    b.step(steps)
    sizes = [int(np.prod(d["shape"])) for d in doms]
    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[1]), int(order[2]), int(np.random.default_rng(9).integers(0, 64))]
    for k in pick:
        d = doms[k]
        _, u_ref, S = oracle_run(d, steps)
        _, u = b.macros(k)
        m = fluid_mask(d)
        err = rel_l2_u(u.double().cpu().numpy(), u_ref, m)
        tot = b.sums(k, 1)[0]
        ref = oracle.sums(S, d["flags"])
        say(f"  domain {k} {d['shape']} tau={d['tau']:.3f}: rel-L2(u) = {err:.3e}, "
            f"mass {abs(tot[0] - ref[0]) / ref[0]:.1e}")
        assert err <= TOL_U["f32"]
        assert abs(tot[0] - ref[0]) <= 1e-8 * ref[0]
    b.close()

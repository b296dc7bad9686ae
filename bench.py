#!/usr/bin/env python3
"""Throughput of the fused D3Q19 BGK step on one MI355X.

Workload: 512^3 periodic lattice, Taylor-Green vortex (u0 = 0.01,
k = 2 pi / 512) plus seeded uniform +-1e-3 noise on every velocity component,
tau = 0.55, no body force; populations stored as FP32, FP16, BF16 or scaled
16-bit fixed point (shifted by the lattice weights), FP32 arithmetic, FP64
conservation totals every step.
A step is one launch of the fused update over all 134,217,728 sites with the
inputs already resident in HBM.

Prints one JSON line: MLUPS of the FP32-storage path as ``value``, the
16-bit-storage results beside it, each codec's error against stored FP64
oracle results of the same workload after 200 and 1000 steps (the
equal-accuracy half of the metric), the HBM roofline of the step kernel
(algorithmic bytes: 19 loads + 19 stores per site), a copy-kernel ceiling
measured in the same run, and the FP64 oracle timed on the host cores on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=512, help="lattice edge (default 512)")
    p.add_argument("--codecs", default="f32,f16,bf16,s16")
    p.add_argument("--no-accuracy", action="store_true",
                   help="skip the 1000-step accuracy leg against the stored oracle results")
    p.add_argument("--cpu-steps", type=int, default=5, help="oracle steps in the CPU baseline sample")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    p.add_argument("--reps", type=int, default=3, help="timed repetitions (median reported)")
    p.add_argument("--no-batch", action="store_true", help="skip the 64-domain batch leg")
    p.add_argument("--batch-steps", type=int, default=500, help="timed steps of the batch leg")
    p.add_argument("--no-adjoint", action="store_true", help="skip the 128^3 force-gradient leg")
    p.add_argument("--no-inplace", action="store_true", help="skip the one-array (in-place) FP32 leg")
    p.add_argument("--no-cavity", action="store_true", help="skip the 4096^2 D2Q9 lid-driven cavity leg")
    p.add_argument("--no-small", action="store_true", help="skip the 32^3 box and 256x128x128 channel legs")
    p.add_argument("--small-steps", type=int, default=0,
                   help="timed steps of the 32^3 box and channel legs (default 0: their own 200 and 5000)")
    return p.parse_args()


def workload_fields(n):
    from paper_2409_16781_amd import inputs
    cfg = inputs.tgv_noise_box(n, u0=0.01, tau=0.55, steps=1000, noise=1e-3, seed=2)
    return cfg


STEP_KERNEL_SOURCES = ("lb_internal.h", "lb_device.h", "lb_kernels.hip")


def step_kernel_digest(root):
    """SHA-256 over the code (comments and whitespace removed) of the sources
    the single-lattice step kernel is built from."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in STEP_KERNEL_SOURCES:
        text = open(os.path.join(root, "paper_2409_16781_amd", "csrc", name)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(codec, n):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counters
    (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a copy of
    known size), or None when the kernel source changed since they were taken
    or the lattice differs."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "step_vec_512cube_tgv.traffic.json")
    try:
        tr = json.load(open(path))
        digest = step_kernel_digest(here)
    except OSError:
        return None
    if n != 512 or tr.get("kernel_source_sha256") != digest:
        return None
    return tr["per_launch_bytes"].get(codec)


def bytes_per_site(codec):
    return 19 * 2 * (4 if codec == "f32" else 2)  # f16, bf16, s16: 2 bytes


def run_codec(torch, lbm, cfg, codec, steps, warmup, reps):
    n = cfg["shape"][0]
    N = n ** 3
    lat = lbm.Lattice(n, n, n, cfg["tau"], codec=codec)
    rho = torch.from_numpy(cfg["rho"]).cuda()
    u = torch.from_numpy(cfg["u"]).cuda()
    lat.init_eq(rho, u)
    del rho, u
    torch.cuda.synchronize()
    log(f"[bench] {codec}: variant={lat.info} warmup={warmup}")
    lat.step(warmup)
    lat.sync()
    extra = 0
    if codec == "s16":
        # scaled 16-bit storage widens a class's range when the first steps'
        # transients outgrow it (the flagged steps are redone): keep warming
        # up, untimed, until ten steps pass without a widening
        while extra < 200:
            w0 = lat.info["rescales"]
            lat.step(10)
            lat.sync()
            extra += 10
            if lat.info["rescales"] == w0:
                break
    widen0 = lat.info["rescales"]
    times = []
    for r in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = lat.time_steps(steps)     # HIP events on the lattice stream around the K launches
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        times.append((ms, wall))
        log(f"[bench] {codec}: rep {r}: {ms:.2f} ms for {steps} steps (wall {wall * 1e3:.2f} ms)")
    # value: the wall clock of exactly `steps` steps between two device
    # synchronisations (median of the repetitions); the HIP-event time of
    # the same launches is reported beside it
    ms_med = sorted(t[0] for t in times)[len(times) // 2]
    wall_med = sorted(t[1] for t in times)[len(times) // 2]
    per_step_ms = wall_med * 1e3 / steps
    mlups = N * steps / wall_med / 1e6
    # dominant kernel alone: HIP events on the lattice stream around each step kernel
    kernel_ms = lat.time_step_kernel(min(steps, 50))
    gbs = bytes_per_site(codec) * N / (kernel_ms * 1e-3) / 1e9
    copy_ms = lat.copy_probe(10)
    copy_bytes = 2 * lat.info["array_bytes"]
    copy_gbs = copy_bytes / (copy_ms * 1e-3) / 1e9
    sums = lat.sums(min(steps, 4096))
    drift = float(abs(sums[-1, 0] - sums[0, 0]) / sums[0, 0])
    r_out, u_out = lat.macros()
    torch.cuda.synchronize()
    res = dict(codec=codec, mlups=mlups, ms_per_step=per_step_ms, wall_ms=wall_med * 1e3, event_ms=ms_med,
               step_kernel_ms=kernel_ms, achieved_gbs=gbs, frac_hbm=gbs / HBM_PEAK_GBS, copy_gbs=copy_gbs,
               frac_copy=gbs / copy_gbs, mass_drift_per_step=drift / max(1, len(sums) - 1),
               variant=lat.info["variant"], sites_per_thread=lat.info["sites_per_thread"],
               grid=lat.info["grid"], steps_done=lat.steps_done)
    if codec == "s16":
        res["exponents"] = [int(e) for e in lat.get_scales()]
        res["widenings_warmup"] = widen0
        res["warmup_steps_added"] = extra
        res["widenings_timed"] = lat.info["rescales"] - widen0
    lat.close()
    return res, u_out


def run_batch(torch, lbm, steps, reps):
    """64 porous channel domains (extents U{16..96}, porosity 0.8, tau
    U[0.55, 1.0], force 1e-6) advanced by one launch per step in the
    autotuned launch shape."""
    from paper_2409_16781_amd import inputs
    doms = inputs.batch_domains(64, seed=3)
    b = lbm.Batch([(d["shape"][2], d["shape"][1], d["shape"][0]) for d in doms], [d["tau"] for d in doms],
                  flags=[d["flags"] for d in doms], codec="f32", autotune=True)
    for k, d in enumerate(doms):
        b.set_force(*d["force"], domain=k)
        b.init_eq(k, torch.from_numpy(d["rho"]).cuda(), torch.from_numpy(d["u"]).cuda())
    info = b.info
    b.step(20)
    b.sync()
    ms = sorted(b.time_steps(steps) for _ in range(reps))[reps // 2]
    kernel_ms = b.time_step_kernel(50)
    fluid, sites = info["fluid_sites"], info["sites"]
    gbs = 152.0 * fluid / (kernel_ms * 1e-3) / 1e9
    sums = b.sums(0, 1)
    b.close()
    return dict(workload="64 D3Q19 porous channel domains, extents U{16..96} per axis (seed 3), walls y=0/ny-1 + "
                         "spheres r~U[2,6] to porosity 0.8, tau~U[0.55,1.0], force 1e-6, FP32 storage",
                domains=64, sites=sites, fluid_sites=fluid, steps=steps, ms_per_step=round(ms, 5),
                mlups_fluid=round(fluid / (ms * 1e-3) / 1e6, 1), mlups_all_sites=round(sites / (ms * 1e-3) / 1e6, 1),
                kernel_ms=round(kernel_ms, 5), achieved_gbs_fluid=round(gbs, 1),
                frac_hbm=round(gbs / HBM_PEAK_GBS, 4), bytes_per_fluid_site=152,
                shape={k: info[k] for k in ("variant", "sites_per_lane", "grid", "tiles", "tile_order", "seg_bytes",
                                             "grid_mult", "autotuned", "wg_cap")},
                finite_totals=bool(np.all(np.isfinite(sums))))


def run_inplace(torch, lbm, cfg, steps, reps):
    """The 512^3 workload with one population array (in-place update, FP32)."""
    n = cfg["shape"][0]
    lat = lbm.Lattice(n, n, n, cfg["tau"], codec="f32", inplace=True)
    lat.init_eq(torch.from_numpy(cfg["rho"]).cuda(), torch.from_numpy(cfg["u"]).cuda())
    torch.cuda.empty_cache()
    lat.step(20)
    lat.sync()
    ms = sorted(lat.time_steps(steps) for _ in range(reps))[reps // 2]
    k_even, k_odd = lat.time_step_kernel(1), lat.time_step_kernel(1)
    info = lat.info
    lat.close()
    return dict(workload="same 512^3 workload, FP32, one population array (in-place update)",
                mlups=round(n ** 3 * steps / (ms * 1e-3) / 1e6, 1), ms_per_step=round(ms / steps, 4),
                kernel_ms_gather_push=round(k_even, 4), kernel_ms_local=round(k_odd, 4),
                array_bytes=info["array_bytes"], arrays=1)


def run_adjoint(torch, lbm, reps):
    """Gradient of the outlet mass flux of a 128^3 porous channel (porosity
    0.85) with respect to the per-site x-force: 500 forward steps with a
    checkpoint every 50, recomputation and 500 adjoint steps (FP32
    storage)."""
    from paper_2409_16781_amd import inputs
    cfg = inputs.porous_channel(128, porosity=0.85, tau=0.6, g=1e-6, seed=4, steps=500, every=50)
    n = 128
    lat = lbm.Lattice(n, n, n, cfg["tau"], flags=cfg["flags"])
    lat.set_force(*cfg["force"])
    fluid = torch.from_numpy(cfg["flags"] == 0).cuda()
    rho = torch.from_numpy(cfg["rho"]).cuda()
    u = torch.from_numpy(cfg["u"]).cuda()
    lat.set_force_field(torch.zeros((n, n, n), dtype=torch.float32, device="cuda"))
    lat.init_eq(rho, u)
    shape = lat.tune(10)  # forward (and recompute) launch shape for this lattice
    lat.grad_outlet_flux_x(cfg["steps"], cfg["every"])  # warm-up: allocates the sweep's buffers
    times = []
    for _ in range(reps):
        lat.init_eq(rho, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, g = lat.grad_outlet_flux_x(cfg["steps"], cfg["every"])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[len(times) // 2]
    fl = int(fluid.sum())
    lat.close()
    return dict(workload="128^3 porous channel (porosity 0.85, seed 4), tau=0.6, force 1e-6, gradient of the outlet "
                         "mass flux w.r.t. the per-site x-force, 500 steps, checkpoints every 50, FP32",
                sites=n ** 3, fluid_sites=fl, steps=cfg["steps"], every=cfg["every"],
                ms_per_gradient=round(dt * 1e3, 3),
                forward_shape={k: shape[k] for k in ("variant", "sites_per_thread", "tile_order", "pull_nt", "grid")},
                site_steps_per_s=round(3 * cfg["steps"] * n ** 3 / dt / 1e6, 1),
                note="forward + recompute + adjoint = 3 x steps site updates; the sweep's buffers are kept by the lattice "
                     "from the warm-up call on",
                finite=bool(torch.isfinite(g).all()))


def run_cavity2d(torch, lbm, steps, reps):
    """The paper's own workload: D2Q9 lid-driven cavity, 4096^2 sites,
    Re = 1e4, lid speed 0.1, FP32 storage of f - w, FP64 totals per step."""
    from paper_2409_16781_amd import inputs
    cfg = inputs.lid_cavity(4096)
    ny, nx = cfg["shape"]
    lat = lbm.Lattice2D(nx, ny, cfg["tau"], flags=cfg["flags"], lid=cfg["lid"])
    lat.init_eq()
    lat.step(50)
    lat.sync()
    ms = sorted(lat.time_steps(steps) for _ in range(reps))[reps // 2]
    sums = lat.sums(min(steps, 1000))
    n = nx * ny
    fluid = int((cfg["flags"] == 0).sum())
    lat.close()
    return dict(workload=f"D2Q9 lid-driven cavity {nx}x{ny}, Re=1e4, lid 0.1, tau={cfg['tau']:.5f}, FP32",
                mlups=round(n * steps / (ms * 1e-3) / 1e6, 1), mlups_fluid=round(fluid * steps / (ms * 1e-3) / 1e6, 1),
                ms_per_step=round(ms / steps, 4), bytes_per_site=72,
                achieved_gbs=round(72 * n * steps / (ms * 1e-3) / 1e9, 1),
                frac_hbm=round(72 * n * steps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                note="time per step includes the FP64 totals (one totals kernel per run of steps)",
                finite_totals=bool(np.all(np.isfinite(sums))))


def run_small(torch, lbm, reps, steps=0):
    """The two smaller D3Q19 workloads at their full step counts, FP32 and
    FP16 storage: the 32^3 Taylor-Green box (200 steps; its 5 MB of state
    stays in the caches, so it is no HBM roofline point) and the
    256 x 128 x 128 force-driven channel (walls at y = 0 and 127, 5000 steps)."""
    from paper_2409_16781_amd import inputs
    out = {}
    for key, cfg in (("tgv32", inputs.tgv_box(32)), ("channel256", inputs.channel())):
        if steps > 0:
            cfg["steps"] = steps
        nz, ny, nx = cfg["shape"]
        n = nx * ny * nz
        entry = dict(workload=f"D3Q19 {cfg['name']}, tau={cfg['tau']}, force={cfg['force'][0]:g}, "
                              f"{cfg['steps']} steps", sites=n, steps=cfg["steps"])
        if cfg["flags"] is not None:
            entry["fluid_sites"] = int((cfg["flags"] == 0).sum())
        for codec in ("f32", "f16"):
            lat = lbm.Lattice(nx, ny, nz, cfg["tau"], flags=cfg["flags"], codec=codec)
            lat.set_force(*cfg["force"])
            rho = torch.from_numpy(cfg["rho"]).cuda()
            u = torch.from_numpy(cfg["u"]).cuda()
            lat.init_eq(rho, u)
            shape = lat.tune(10)  # launch shape for this lattice (state unchanged)
            lat.step(64)  # warm-up
            times = []
            for _ in range(reps):
                lat.init_eq(rho, u)
                lat.sync()
                times.append(lat.time_steps(cfg["steps"]))
            ms = sorted(times)[reps // 2]
            kernel_ms = lat.time_step_kernel(50)
            sums = lat.sums(1)
            lat.close()
            nf = entry.get("fluid_sites", n)  # algorithmic bytes: fluid sites only
            kgbs = bytes_per_site(codec) * nf / (kernel_ms * 1e-3) / 1e9
            gbs = bytes_per_site(codec) * nf * cfg["steps"] / (ms * 1e-3) / 1e9
            # kernel_ms: HIP events around single eagerly launched kernels,
            # which on steps of tens of microseconds include a few
            # microseconds of launch; the step rate of the captured run
            # (gbs_algorithmic, frac_hbm) carries no such overhead
            entry[codec] = dict(mlups=round(n * cfg["steps"] / (ms * 1e-3) / 1e6, 1),
                                ms_per_step=round(ms / cfg["steps"], 5),
                                gbs_algorithmic=round(gbs, 1), frac_hbm=round(gbs / HBM_PEAK_GBS, 4),
                                kernel_ms=round(kernel_ms, 5), kernel_gbs=round(kgbs, 1),
                                kernel_frac_hbm=round(kgbs / HBM_PEAK_GBS, 4),
                                shape={k: shape[k] for k in ("variant", "sites_per_thread", "tile_order", "pull_nt", "grid")},
                                finite_totals=bool(np.all(np.isfinite(sums))))
        out[key] = entry
    return out


GOLDEN_NOISE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                            "tgv512_noise_golden.npz")
ACCURACY_BOUND = {"f32": 1e-5, "f16": 2e-3, "bf16": 2e-3, "s16": 2e-3}


def accuracy_vs_oracle(torch, lbm, cfg, codecs):
    """rel-L2 of u against stored FP64 oracle results of the same 512^3
    workload (written by tests/golden/make_tgv512_noise_golden.py from the
    oracle alone) at their seeded sample sites, after 200 and 1000 steps."""
    n = cfg["shape"][0]
    if n != 512 or not os.path.exists(GOLDEN_NOISE):
        return None
    with np.load(GOLDEN_NOISE) as z:
        gold = {k: z[k] for k in z.files}
    idx = torch.from_numpy(gold["sites_zyx"]).cuda()
    out = {}
    for codec in codecs:
        lat = lbm.Lattice(n, n, n, cfg["tau"], codec=codec)
        lat.init_eq(torch.from_numpy(cfg["rho"]).cuda(), torch.from_numpy(cfg["u"]).cuda())
        torch.cuda.empty_cache()
        res, done = {}, 0
        for k in (200, 1000):
            lat.step(k - done)
            done = k
            _, u = lat.macros()
            ug = u[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.double().cpu().numpy()
            ref = gold[f"u_{k}"]
            res[f"rel_l2_u_{k}"] = float(np.linalg.norm(ug - ref) / np.linalg.norm(ref))
            del u
        res["bound"] = ACCURACY_BOUND.get(codec)
        res["meets_bound"] = bool(res["rel_l2_u_1000"] <= res["bound"])
        if codec == "s16":
            res["exponents"] = [int(e) for e in lat.get_scales()]
            res["widenings"] = lat.info["rescales"]
        lat.close()
        torch.cuda.empty_cache()
        out[codec] = res
        log(f"[bench] accuracy {codec}: rel-L2(u) vs oracle {res['rel_l2_u_200']:.2e} (200 steps), "
            f"{res['rel_l2_u_1000']:.2e} (1000 steps), bound {res['bound']:g}")
    out["samples"] = int(len(gold["sites_zyx"]))
    out["reference"] = "FP64 oracle, tests/golden/tgv512_noise_golden.npz"
    return out


def cpu_baseline(cfg, steps):
    """The FP64 oracle as it stands, on the host cores, for a few steps of the same lattice."""
    import oracle
    oracle.build(force=False)
    n = cfg["shape"][0]
    S = oracle.init(cfg["shape"], cfg["rho"], cfg["u"], None)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    S = oracle.run(S, cfg["tau"], steps)
    dt = time.perf_counter() - t0
    del S
    return dict(value=n ** 3 * steps / dt / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{n}^3 lattice of the same workload, {steps} FP64 steps, {dt:.1f} s",
                cpu_model=cpu_model(), nproc=os.cpu_count())


def cpu_model():
    """The host CPU's model name, with its family and model numbers (from
    /proc/cpuinfo: a virtual machine may report a short name); None where it
    is absent."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # the first processor's block is enough
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    except OSError:
        return None
    name = fields.get("model name")
    if name is None:
        return None
    extra = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    return f"{name} ({', '.join(extra)})" if extra else name


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the step of one lattice on one device); --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_2409_16781_amd as lbm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    n = args.n
    log(f"[bench] generating {n}^3 Taylor-Green + noise inputs")
    cfg = workload_fields(n)
    results = {}
    u_fields = {}
    for codec in args.codecs.split(","):
        res, u = run_codec(torch, lbm, cfg, codec, args.steps, args.warmup, args.reps)
        results[codec] = res
        u_fields[codec] = u
        log(f"[bench] {codec}: {res['mlups']:.0f} MLUPS, {res['achieved_gbs']:.0f} GB/s "
            f"({100 * res['frac_hbm']:.1f}% of HBM peak, {100 * res['frac_copy']:.1f}% of copy)")
    # FP16 / BF16 vs FP32 after the same number of steps (GPU vs GPU, not parity)
    if "f32" in u_fields:
        ref = u_fields["f32"].double()
        for c in u_fields:
            if c != "f32":
                d = (u_fields[c].double() - ref).norm() / ref.norm()
                results[c]["rel_l2_u_vs_f32"] = float(d)
    del u_fields
    torch.cuda.empty_cache()

    main_codec = "f32" if "f32" in results else list(results)[0]
    m = results[main_codec]
    N = n ** 3
    traffic_bytes = measured_traffic(main_codec, n)
    traffic_gbs = None if traffic_bytes is None else traffic_bytes / (m["step_kernel_ms"] * 1e-3) / 1e9
    line = {
        "metric": "D3Q19 MLUPS & % HBM peak at 512³: FP32 vs FP16-store, equal-accuracy",
        "value": round(m["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q19 BGK periodic {n}^3 Taylor-Green (u0=0.01) + seeded U(+-1e-3) "
                               f"velocity noise, tau=0.55, {main_codec} storage, FP64 GPU totals per step",
                   "sites": N, "storage": main_codec, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(m["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(m["frac_hbm"], 4),
                     "traffic": None if traffic_gbs is None else round(traffic_gbs, 1),
                     "traffic_bytes_per_launch": traffic_bytes,
                     "traffic_bytes_per_site": None if traffic_bytes is None else round(traffic_bytes / N, 2),
                     "bytes_per_site": bytes_per_site(main_codec), "kernel_ms": round(m["step_kernel_ms"], 4),
                     "kernel": "step_vec (fused pull-stream + BGK/Guo collide)",
                     "copy_ceiling_gbs": round(m["copy_gbs"], 1), "frac_of_copy": round(m["frac_copy"], 4)},
        "variants": {c: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
                     for c, r in results.items()},
    }
    if "f16" in results and "f32" in results:
        line["f16_over_f32_mlups"] = round(results["f16"]["mlups"] / results["f32"]["mlups"], 3)
    if "s16" in results and "f32" in results:
        line["s16_over_f32_mlups"] = round(results["s16"]["mlups"] / results["f32"]["mlups"], 3)
    if not args.no_accuracy:
        log("[bench] accuracy against the stored FP64 oracle results (1000 steps per codec)")
        acc = accuracy_vs_oracle(torch, lbm, cfg, list(results))
        if acc is not None:
            line["accuracy_vs_oracle"] = acc
    if not args.no_inplace and n == 512:
        log("[bench] one-array (in-place) FP32")
        line["inplace_f32"] = run_inplace(torch, lbm, cfg, args.steps, args.reps)
        log(f"[bench] in-place f32: {line['inplace_f32']['mlups']:.0f} MLUPS")
    if not args.no_batch:
        log("[bench] batch of 64 porous domains (autotuned)")
        line["batch64"] = run_batch(torch, lbm, args.batch_steps, args.reps)
        log(f"[bench] batch64: {line['batch64']['mlups_fluid']:.0f} fluid MLUPS, "
            f"{line['batch64']['achieved_gbs_fluid']:.0f} GB/s")
    if not args.no_adjoint:
        log("[bench] adjoint: 128^3 porous force gradient")
        line["adjoint128"] = run_adjoint(torch, lbm, args.reps)
        log(f"[bench] adjoint128: {line['adjoint128']['ms_per_gradient']:.1f} ms per gradient")
    if not args.no_cavity:
        log("[bench] D2Q9 4096^2 lid-driven cavity")
        line["cavity4096_d2q9"] = run_cavity2d(torch, lbm, 2 * args.steps, args.reps)
        log(f"[bench] cavity4096: {line['cavity4096_d2q9']['mlups']:.0f} MLUPS, "
            f"{line['cavity4096_d2q9']['achieved_gbs']:.0f} GB/s")
    if not args.no_small:
        log("[bench] 32^3 Taylor-Green box and 256x128x128 channel, full step counts")
        line.update(run_small(torch, lbm, args.reps, args.small_steps))
        for k in ("tgv32", "channel256"):
            log(f"[bench] {k}: f32 {line[k]['f32']['mlups']:.0f} MLUPS, f16 {line[k]['f16']['mlups']:.0f} MLUPS")
    if not args.no_cpu:
        log(f"[bench] CPU baseline: oracle, {args.cpu_steps} steps")
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

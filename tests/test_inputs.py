"""The seeded input generators (shared by the oracle runs and the GPU runs):
reproducible, with the geometry and statistics their workloads state.  CPU only."""
import math

import numpy as np

from paper_2409_16781_amd import inputs


def test_noise_is_seeded_uniform_and_bounded():
    a = inputs.uniform_noise((4, 5, 6), 1e-3, 7)
    assert np.array_equal(a, inputs.uniform_noise((4, 5, 6), 1e-3, 7))
    assert not np.array_equal(a, inputs.uniform_noise((4, 5, 6), 1e-3, 8))
    assert np.abs(a).max() <= 1e-3
    big = inputs.uniform_noise((200000,), 1.0, 1)
    assert abs(big.mean()) < 0.01 and abs(big.var() - 1.0 / 3.0) < 0.01   # U(-1, 1)


def test_taylor_green_fields_are_divergence_free_and_z_uniform():
    rho, u = inputs.tgv_fields(16, 16, 4, 0.01)
    assert u.shape == (3, 4, 16, 16) and np.all(u[2] == 0.0)
    assert np.array_equal(u[:, 0], u[:, 3]) and np.array_equal(rho[0], rho[3])
    # spectral divergence of the periodic field vanishes
    k = 2 * np.pi * np.fft.fftfreq(16)
    div = 1j * k[None, :] * np.fft.fft2(u[0, 0]) + 1j * k[:, None] * np.fft.fft2(u[1, 0])
    assert np.abs(div).max() < 1e-12
    assert abs(u[0].max() - 0.01) < 1e-3


def test_channel_and_cavity_geometry():
    f = inputs.channel_flags(8, 6, 3)
    assert np.all(f[:, 0, :] == 1) and np.all(f[:, -1, :] == 1) and np.all(f[:, 1:-1, :] == 0)
    c = inputs.cavity_flags(7, 5)
    assert np.all(c[0] == 1) and np.all(c[:, 0] == 1) and np.all(c[:, -1] == 1)
    assert np.all(c[-1, 1:-1] == 2) and c[-1, 0] == 1 and c[-1, -1] == 1
    assert np.all(c[1:-1, 1:-1] == 0)


def test_paper_cavity_parameters():
    cfg = inputs.lid_cavity(4096)
    nu = 0.1 * 4094 / 1e4
    assert abs(cfg["tau"] - (3 * nu + 0.5)) < 1e-15
    assert abs(cfg["tau"] - 0.62282) < 1e-5
    assert cfg["lid"] == (0.1, 0.0) and cfg["shape"] == (4096, 4096)


def test_sphere_packing_reaches_porosity_and_is_seeded():
    f = inputs.sphere_flags(48, 40, 32, 0.8, 3, rmin=2.0, rmax=6.0, walls=True)
    assert np.array_equal(f, inputs.sphere_flags(48, 40, 32, 0.8, 3, rmin=2.0, rmax=6.0, walls=True))
    porosity = (f == 0).mean()
    assert 0.75 <= porosity <= 0.8 + 1e-9
    assert np.all(f[:, 0, :] == 1) and np.all(f[:, -1, :] == 1)
    assert set(np.unique(f)) <= {0, 1}


def test_batch_workload_recipe():
    doms = inputs.batch_domains(64, seed=3)
    assert len(doms) == 64
    dims = np.array([d["shape"] for d in doms])
    assert dims.min() >= 16 and dims.max() <= 96
    taus = np.array([d["tau"] for d in doms])
    assert taus.min() >= 0.55 and taus.max() <= 1.0
    assert all(d["force"] == (1e-6, 0.0, 0.0) for d in doms)
    assert all(np.abs(d["rho"] - 1.0).max() <= 1e-4 for d in doms)
    again = inputs.batch_domains(64, seed=3)
    assert all(np.array_equal(a["flags"], b["flags"]) for a, b in zip(doms, again))


def test_porous_channel_recipe():
    cfg = inputs.porous_channel(48, porosity=0.85, seed=4)
    por = (cfg["flags"] == 0).mean()
    assert 0.8 <= por <= 0.85 + 1e-9
    assert np.all(cfg["rho"] == 1.0) and np.all(cfg["u"] == 0.0)
    assert cfg["force"] == (1e-6, 0.0, 0.0) and cfg["every"] == 50 and cfg["steps"] == 500
    assert math.isclose(cfg["tau"], 0.6)

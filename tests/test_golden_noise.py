"""CPU checks of the stored FP64 oracle results of the 512^3 Taylor-Green +
noise workload (tests/golden/tgv512_noise_golden.*), against what the method
fixes independently of the oracle:

* the amplitude of the initial Taylor-Green mode decays as exp(-2 nu k^2 t)
  with nu = (tau - 1/2) / 3 (the vortex's viscous decay, Section 3.3's test
  case; the U(+-1e-3) noise projects on the mode only at O(noise / sqrt(N)));
* periodic BGK conserves mass and momentum exactly: the stored totals at 0,
  200 and 1000 steps agree to the rounding of an FP64 sum over 2.5e9 values;
* the stored samples are the seeded sites the generator states, with finite
  values of the right magnitude.
"""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
BASE = os.path.join(HERE, "golden", "tgv512_noise_golden")

pytestmark = pytest.mark.skipif(not os.path.exists(BASE + ".npz"), reason="stored 512^3 oracle results missing")


@pytest.fixture(scope="module")
def golden():
    with open(BASE + ".json") as f:
        meta = json.load(f)
    with np.load(BASE + ".npz") as z:
        arr = {k: z[k] for k in z.files}
    return meta, arr


def test_mode_amplitude_decays_at_the_viscous_rate(golden):
    meta, _ = golden
    nu = (0.55 - 0.5) / 3.0
    k = 2.0 * math.pi / 512
    a0 = meta["initial"]["mode_amplitude"]
    assert abs(a0 - 0.01) <= 1e-5  # u0 = 0.01 plus the noise's projection
    for n in (200, 1000):
        a = meta["checkpoints"][str(n)]["mode_amplitude"]
        expect = a0 * math.exp(-2.0 * nu * k * k * n)
        assert abs(a / expect - 1.0) <= 1e-4, (n, a, expect)


def test_mass_and_momentum_are_conserved(golden):
    meta, _ = golden
    s0 = np.array(meta["initial_sums"])
    n_sites = 512 ** 3
    for n in (200, 1000):
        s = np.array(meta["checkpoints"][str(n)]["sums"])
        # FP64 sums over 19 * 512^3 values: rounding ~ 1e-12 of the mass
        assert abs(s[0] - s0[0]) <= 1e-11 * n_sites, (n, s[0], s0[0])
        assert np.all(np.abs(s[1:] - s0[1:]) <= 1e-8), (n, s[1:], s0[1:])
    assert abs(s0[0] - n_sites) <= 1e-3  # mean density 1 (the noise is on u only)


def test_samples_are_the_seeded_sites(golden):
    meta, arr = golden
    sites = arr["sites_zyx"]
    assert sites.shape == (meta["samples"], 3) and sites.min() >= 0 and sites.max() < 512
    rng = np.random.default_rng(meta["sample_seed"])
    lin = np.sort(rng.choice(512 ** 3, size=meta["samples"], replace=False))
    assert np.array_equal(lin, (sites[:, 0] * 512 + sites[:, 1]) * 512 + sites[:, 2])
    for n in (200, 1000):
        u, rho = arr[f"u_{n}"], arr[f"rho_{n}"]
        assert u.shape == (meta["samples"], 3) and rho.shape == (meta["samples"],)
        assert np.all(np.isfinite(u)) and np.abs(u).max() <= meta["checkpoints"][str(n)]["max_abs_u"]
        assert np.abs(rho - 1.0).max() < 1e-3

"""The seeded input generators: determinism, shapes and the set-up recipes."""
import math

import numpy as np

from paper_2005_12764_amd import workloads as W


def test_generators_are_deterministic():
    a = W.single_droplet(seed=3)
    b = W.single_droplet(seed=3)
    c = W.single_droplet(seed=4)
    assert np.array_equal(a.rho_r, b.rho_r) and np.array_equal(a.rho_b, b.rho_b)
    assert not np.array_equal(a.rho_r, c.rho_r)


def test_single_droplet_recipe():
    w = W.single_droplet(seed=0)
    assert w.shape == (32, 32, 32) and w.steps == 200
    rho = w.rho_r + w.rho_b
    assert np.abs(rho - 1).max() <= 1e-4                    # density noise +-1e-4
    phi = (w.rho_r - w.rho_b) / rho
    assert np.allclose(phi, phi[::-1, ::-1, ::-1], atol=1e-12)   # mirror-symmetric droplet
    assert math.isclose(phi[15, 15, 15], math.tanh((8 - math.sqrt(3) / 2) / 2), rel_tol=1e-12)


def test_emulsion_reaches_volume_fraction_without_overlap():
    rng = np.random.default_rng(0)
    n = (96, 96, 96)
    cen, rad, info = W.emulsion(rng, n, 0.30, 6.0, 12.0)
    assert info["inflate"] == 1.0 and abs(info["rsa_phi_v"] - 0.30) < 0.02
    d = cen[:, None, :] - cen[None, :, :]
    d -= np.array(n) * np.round(d / np.array(n))
    dist = np.sqrt((d ** 2).sum(-1)) + np.eye(len(rad)) * 1e9
    assert np.all(dist >= rad[:, None] + rad[None, :] + 1.0 - 1e-9)
    assert rad.min() >= 6.0 and rad.max() <= 12.0


def test_crystal_channel_layout():
    w = W.crystal_channel(seed=1)
    assert w.shape == (64, 128, 512) and w.info["n_droplets"] == 138
    assert tuple(w.params["bc"]) == (0, 1, 1) and w.params["body_force"][0] == 1e-6


def test_job_stream_ranges():
    jobs = W.job_stream(seed=0, n_jobs=200)
    t = np.array([j.arrival for j in jobs])
    assert np.all(np.diff(t) > 0)
    assert 25 < len(jobs) / t[-1] < 60                      # ~40 jobs/s
    assert {j.side for j in jobs} <= {32, 48, 64, 96, 128}
    assert all(0.6 <= j.tau <= 1.2 and 0.002 <= j.A <= 0.02 and 0 <= j.nc_strength <= 0.05
               for j in jobs)

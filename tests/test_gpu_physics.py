"""Physics of the GPU path in every storage form.

- plane Poiseuille flow (walls in y, body force along x) at tau = 1/2 + sqrt(3)/4,
  where halfway bounce-back with the exact-difference force reproduces the
  parabola to round-off: relative L2 error of the physical velocity
  (j + F/2)/rho against u(y) = g/(2 nu) (y + 1/2)(H - 1/2 - y);
  gates: FP64 1e-10, FP32 1e-4, fp16 moment-split 1e-3, bf16 5e-3;
- Laplace's law for static 3-D droplets R = 10, 12, 16: the pressure jump
  p_in - p_out (p = rho/3) of every storage form within 2 % of 2 sigma / R with
  sigma = 2 A tau / 9, and each 16-bit jump within 2 % of the FP32 jump;
- the microfluidic-crystal channel (walls, body force, near-contact) in FP32
  and 16-bit against the FP64 GPU run with the same |G| threshold.
"""
import math

import numpy as np
import pytest

from paper_2005_12764_amd import lb
from paper_2005_12764_amd import workloads as W
from tests.helpers import state_errors

pytestmark = pytest.mark.gpu

POIS_TOL = {W.F64: 1e-10, W.F32: 1e-4, W.F16: 1e-3, W.BF16: 5e-3}


@pytest.mark.parametrize("storage", [W.F64, W.F32, W.F16, W.BF16])
def test_poiseuille_channel(storage):
    H, g = 32, 1e-6
    tau = 0.5 + math.sqrt(3) / 4
    nu = (tau - 0.5) / 3
    w = W.channel(H=H, nx=4, nz=4, force=g, tau=tau, storage=storage)
    with lb.Lattice(dict(w.params, storage=storage)) as L:
        L.init(w.rho_r, w.rho_b)
        L.step(int(8 * H * H / nu))
        rr, rb, j = L.moments()
    ux = ((j[0] + g / 2) / (rr + rb)).mean(axis=(0, 2))
    y = np.arange(H)
    ua = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    err = float(np.linalg.norm(ux - ua) / np.linalg.norm(ua))
    print("poiseuille storage=%d L2 error %.3e" % (storage, err), flush=True)
    assert err <= POIS_TOL[storage]


def _pressure_jump(storage, R, n=48, A=0.01, tau=1.0, steps=3000):
    w = W.sphere(n=n, R=R, A=A, tau=tau, storage=storage)
    with lb.Lattice(dict(w.params, storage=storage)) as L:
        L.init(w.rho_r, w.rho_b).step(steps)
        rr, rb, _ = L.moments()
    rho, phi = rr + rb, (rr - rb) / (rr + rb)
    c = (n - 1) / 2
    z, y, x = np.mgrid[0:n, 0:n, 0:n]
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    Rm = (3 * (phi > 0).sum() / (4 * math.pi)) ** (1 / 3)
    return Rm, (rho[r < Rm - 3].mean() - rho[r > Rm + 3].mean()) / 3.0


def test_laplace_law_all_storage():
    # dp = 2 sigma / R with sigma = 2 A tau / 9 for this perturbation operator:
    # each storage form within 2 % of the law at every radius (radius measured
    # from the droplet volume), and each 16-bit jump within 2 % of FP32's
    # (radii 10-16: the interface, a few sites wide, adds corrections of
    # order width / R to the sharp-interface law)
    A, tau = 0.01, 1.0
    sigma = 2 * A * tau / 9
    radii = (10, 12, 16)
    res = {}
    for storage in (W.F32, W.F16, W.BF16):
        for R in radii:
            Rm, dp = _pressure_jump(storage, R, n=64, A=A, tau=tau)
            res[storage, R] = dp * Rm / (2 * sigma) - 1, dp
            print("laplace storage=%d R=%d Rm %.3f dp %.4e: dp R / (2 sigma) - 1 = %+.2e"
                  % (storage, R, Rm, dp, res[storage, R][0]), flush=True)
    for (storage, R), (law, dp) in res.items():
        assert abs(law) <= 0.02
        assert abs(dp / res[W.F32, R][1] - 1) <= 0.02


def test_crystal_channel_against_fp64():
    # One |G| threshold for every run: below it n = 0 and neither the
    # perturbation nor the recolouring acts.  At a saddle of phi inside a
    # film between two droplets G -> 0 while rho_r rho_b stays large, so the
    # recolouring direction G/|G| is decided by the threshold; runs with
    # different thresholds follow different dynamics there.
    w = W.crystal_channel(seed=0, steps=400)
    out = {}
    for storage in (W.F64, W.F32, W.F16, W.BF16):
        with lb.Lattice(dict(w.params, storage=storage, eps_g=1e-6)) as L:
            L.init(w.rho_r, w.rho_b).step(w.steps)
            out[storage] = L.state()
    # The gates follow from that conditioning, not from the storage: FP32
    # rounds G by ~5e-8, which at a saddle with |G| ~ 1e-6 turns the
    # recolouring direction by a few per cent, i.e. ~1e-3 of a population
    # locally; FP32 and fp16 storage measured alike (~2e-4 after 400 steps),
    # while an FP64 run perturbed by 1e-12 stays at 1e-12.
    for storage, tol in ((W.F32, 5e-4), (W.F16, 5e-4), (W.BF16, 5e-3)):
        e = state_errors(out[storage], out[W.F64])
        print("crystal channel %d steps storage=%d vs fp64: %s" % (w.steps, storage, e), flush=True)
        assert e["worst"] <= tol

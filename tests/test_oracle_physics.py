"""Physics pins of the whole oracle step against textbook results.

- plane Poiseuille flow between halfway bounce-back walls: with BGK and the
  exact-difference forcing the discrete steady state is the analytic parabola
  u(y) = g/(2 nu) (y + 1/2)(H - 1/2 - y) to round-off at tau = 1/2 + sqrt(3)/4,
  and second-order accurate at other tau (Sec. 2 eq:eq1 to eq:eq3, Sec. 2.1
  eq:edm);
- rectangular-duct flow (walls in y and z, force along x): the discrete
  steady state converges at second order to the Fourier-series solution of
  the duct (the corners keep it from being exact at the magic tau);
- a shear wave decays at nu k^2 with the mixture viscosity of Sec. 2.1
  eq:twobgk (harmonic mean weighted by the component densities);
- Laplace's law for a static disc: the pressure jump times the radius is
  constant and matches sigma = 2 A tau / 9 of the perturbation operator;
- near-contact (Sec. 4): droplets at a thin gap merge when N_c = A dx/sigma
  << 1 and stay apart when N_c is of order one or larger.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_12764_amd import workloads as W
from tests.helpers import duct_series, oracle_params


def _poiseuille(H, tau, g, steps):
    w = W.channel(H=H, force=g, tau=tau)
    prm = oracle_params(w.params)
    f = O.init(prm, w.rho_r, w.rho_b)
    f = O.step(prm, f, steps)
    rr, rb, j = O.moments(prm, f)
    ux = ((j[0] + g / 2) / (rr + rb))[0, :, 0]          # physical velocity (j + F/2)/rho
    nu = (tau - 0.5) / 3
    y = np.arange(H)
    ua = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    return float(np.linalg.norm(ux - ua) / np.linalg.norm(ua)), ux, ua


def test_poiseuille_exact_at_magic_tau():
    tau = 0.5 + math.sqrt(3) / 4
    H = 16
    nu = (tau - 0.5) / 3
    err, ux, ua = _poiseuille(H, tau, 1e-6, int(20 * H * H / nu))
    assert err < 1e-10
    assert np.allclose(ux, ux[::-1], rtol=1e-12)        # symmetric about the mid-plane


def _duct(a, b, tau, g=1e-6):
    nu = (tau - 0.5) / 3
    p = W.base_params(2, a, b, bc=(0, 1, 1), storage=W.F64, tau_r=tau, tau_b=tau, body_force=(g, 0.0, 0.0))
    rr = np.ones((b, a, 2))
    prm = oracle_params(p)
    steps = int(36 * b * b / (nu * math.pi ** 2))       # the slowest mode decays by e^-36
    f = O.step(prm, O.init(prm, rr, np.zeros_like(rr)), steps)
    r1, r2, j = O.moments(prm, f)
    ux = ((j[0] + g / 2) / (r1 + r2))[:, :, 0]
    y = np.arange(a) - (a - 1) / 2
    z = np.arange(b) - (b - 1) / 2
    ua = duct_series(a, b, y[None, :], z[:, None], g, nu)
    return float(np.linalg.norm(ux - ua) / np.linalg.norm(ua))


def test_duct_flow_converges_to_the_fourier_series():
    tau = 0.5 + math.sqrt(3) / 4
    e1, e2 = _duct(16, 8, tau), _duct(32, 16, tau)
    assert e1 < 3e-3 and e2 < 6e-4
    assert 3.5 < e1 / e2 < 5.5                          # second order in the cross-section


def test_poiseuille_second_order_at_unit_tau():
    e1, _, _ = _poiseuille(8, 1.0, 1e-6, 4000)
    e2, _, _ = _poiseuille(16, 1.0, 1e-6, 16000)
    assert e1 < 1e-2 and e2 < e1
    assert 3.0 < e1 / e2 < 5.0                          # error falls ~4x when H doubles


@pytest.mark.parametrize("tr,tb,red", [(1.0, 1.0, 1.0), (0.7, 1.3, 0.3), (0.7, 1.3, 0.8),
                                       (1.2, 0.6, 0.5)])
def test_shear_wave_decays_with_mixture_viscosity(tr, tb, red):
    L = 64
    w = W.shear_wave(L=L, U=1e-4, tau_r=tr, tau_b=tb, red_fraction=red)
    prm = oracle_params(w.params)
    f = O.init(prm, w.rho_r, w.rho_b, w.u)
    a0 = np.abs(O.moments(prm, f)[2][0]).max()
    n = 600
    f = O.step(prm, f, n)
    a1 = np.abs(O.moments(prm, f)[2][0]).max()
    k = 2 * math.pi / L
    nubar = 1.0 / (red / ((tr - 0.5) / 3) + (1 - red) / ((tb - 0.5) / 3))
    nu_meas = -math.log(a1 / a0) / n / k ** 2
    assert abs(nu_meas / nubar - 1) < 1e-2       # other readings of the mixture rule are off by >10%


def _disc_pressure_jump(R, A, tau, steps=3000, n=48):
    w = W.disc(n=n, R=R, A=A, tau=tau)
    prm = oracle_params(w.params)
    f = O.step(prm, O.init(prm, w.rho_r, w.rho_b), steps)
    rr, rb, j = O.moments(prm, f)
    rho, phi = (rr + rb)[0], ((rr - rb) / (rr + rb))[0]
    c = (n - 1) / 2
    yy, xx = np.mgrid[0:n, 0:n]
    r = np.hypot(xx - c, yy - c)
    Rm = math.sqrt((phi > 0).sum() / math.pi)            # radius from the measured area
    dp = (rho[r < Rm - 3].mean() - rho[r > Rm + 3].mean()) / 3.0   # p = c_s^2 rho
    return Rm, dp, float(np.abs(j).max())


def test_laplace_law_disc():
    A, tau = 0.01, 1.0
    res = [_disc_pressure_jump(R, A, tau) for R in (8, 10, 12)]
    sig = [dp * Rm for Rm, dp, _ in res]                 # 2D: dp = sigma / R
    assert max(sig) / min(sig) < 1.04
    assert all(abs(s / (2 * A * tau / 9) - 1) < 0.05 for s in sig)
    assert all(um < 1e-4 for _, _, um in res)            # spurious currents stay small


def test_surface_tension_scales_with_A():
    _, dp1, _ = _disc_pressure_jump(10, 0.005, 1.0, steps=2500)
    _, dp2, _ = _disc_pressure_jump(10, 0.010, 1.0, steps=2500)
    assert 1.9 < dp2 / dp1 < 2.1


def _film_midpoint(nc_strength, steps=1500):
    w = W.two_droplets(n=(48, 32, 1), R=8, gap=2.0, A=0.01, nc_strength=nc_strength,
                       nc_range=2, nc_hmin=2.0)
    prm = oracle_params(w.params)
    f = O.step(prm, O.init(prm, w.rho_r, w.rho_b), steps)
    rr, rb, j = O.moments(prm, f)
    phi = (rr - rb) / (rr + rb)
    return float(phi[0, 15:17, 23:25].mean()), j


def test_near_contact_merging_regimes():
    sigma = 2 * 0.01 * 1.0 / 9
    mid_off, _ = _film_midpoint(0.0)
    mid_weak, _ = _film_midpoint(0.1 * sigma)            # N_c = 0.1
    mid_strong, j = _film_midpoint(9.0 * sigma)          # N_c = 9
    assert mid_off > 0.9 and mid_weak > 0.9              # the film drains: droplets merged
    assert mid_strong < -0.9                             # film stabilised, no merging
    assert np.abs(j.sum(axis=(1, 2, 3))).max() < 1e-12   # mirror-symmetric pair: no net push


def test_couette_flow_between_sliding_walls():
    # walls at y = -1/2 and H - 1/2 sliding at -U and +U along x (the sheared
    # channel of Sec. 5): the steady profile is exactly linear, for a mixture too
    H, U = 16, 0.01
    for red in (1.0, 0.4):
        w = W.shear_wave(L=H, U=0.0, tau_r=0.8, tau_b=1.1, red_fraction=red)
        p = dict(w.params, bc=(0, 1, 0))
        p["wall_velocity"] = ((0, 0, 0), (0, 0, 0), (-U, 0, 0), (U, 0, 0), (0, 0, 0), (0, 0, 0))
        prm = oracle_params(p)
        f = O.step(prm, O.init(prm, w.rho_r, w.rho_b), 6000)
        rr, rb, j = O.moments(prm, f)
        ux = (j[0] / (rr + rb))[0, :, 0]
        y = np.arange(H)
        ua = -U + 2 * U * (y + 0.5) / H
        assert np.abs(ux - ua).max() < 1e-12
        r0, b0, _ = O.moments(prm, O.init(prm, w.rho_r, w.rho_b))
        assert abs(rr.sum() / r0.sum() - 1) < 1e-12 and (red == 1.0 or abs(rb.sum() / b0.sum() - 1) < 1e-12)


def test_sliding_walls_conserve_colour_with_droplets():
    w = W.two_droplets(n=(40, 20, 8), R=5, gap=3.0, A=0.01)
    p = dict(w.params, bc=(0, 1, 0))
    p["wall_velocity"] = ((0, 0, 0), (0, 0, 0), (-0.01, 0, 0), (0.01, 0, 0), (0, 0, 0), (0, 0, 0))
    prm = oracle_params(p)
    f0 = O.init(prm, w.rho_r, w.rho_b)
    f = O.step(prm, f0, 200)
    r0, b0, _ = O.moments(prm, f0)
    r1, b1, j1 = O.moments(prm, f)
    assert abs(r1.sum() / r0.sum() - 1) < 1e-12 and abs(b1.sum() / b0.sum() - 1) < 1e-12
    # the walls drag the fluid: positive x-momentum near the top wall, negative near the bottom
    assert j1[0][:, -1, :].mean() > 0 > j1[0][:, 0, :].mean()

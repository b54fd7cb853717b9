"""Pins of the oracle's per-site pieces against closed forms.

Each check follows from the mathematics of the pieces, not from re-typing
them: moment identities of the D3Q19 set and the equilibrium (Sec. 2,
eq:equil, eq:eq2), the exact-difference source (Sec. 2.1, eq:edm), the mixture
relaxation rate (Sec. 2.1, eq:twobgk with eq:eq3), the moments of the
colour-gradient perturbation and of recolouring, and the near-contact
amplitude A_h (Sec. 4).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

RNG = np.random.default_rng(1234)
I3 = np.eye(3)


def _tables():
    c, w, opp, bp = O.tables()
    return c.astype(np.float64), w, opp, bp


# --------------------------------------------------------------- lattice (U1)

def test_d3q19_lattice_isotropy():
    c, w, opp, bp = _tables()
    assert len({tuple(v) for v in c.astype(int)}) == 19
    assert np.all(np.abs(c) <= 1) and np.all((c ** 2).sum(1) <= 2)
    assert math.isclose(w.sum(), 1.0, abs_tol=1e-15)                       # normalised
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), I3 / 3, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", I3, I3) + np.einsum("ac,bd->abcd", I3, I3)
           + np.einsum("ad,bc->abcd", I3, I3)) / 9.0
    assert np.allclose(m4, iso, atol=1e-16)
    for i in range(19):
        assert np.array_equal(c[opp[i]], -c[i])
        assert opp[opp[i]] == i
    # perturbation coefficients: zero total mass and first moment, isotropic second
    assert math.isclose(bp.sum(), 1.0 / 3.0, abs_tol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", bp, c, c), I3 / 3, atol=1e-16)


# ---------------------------------------------------------- equilibrium (U2)

@pytest.mark.parametrize("trial", range(5))
def test_equilibrium_moments(trial):
    c, w, _, _ = _tables()
    rho = RNG.uniform(0.2, 2.0)
    u = RNG.uniform(-0.1, 0.1, 3)
    f = O.feq(rho, u)
    assert math.isclose(f.sum(), rho, rel_tol=1e-14)
    assert np.allclose(f @ c, rho * u, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", f, c, c), rho * (I3 / 3 + np.outer(u, u)),
                       atol=1e-15)


def test_equilibrium_at_rest_is_the_weights():
    _, w, _, _ = _tables()
    assert np.array_equal(O.feq(1.0, [0, 0, 0]), w)


# ---------------------------------------------------- mixture relaxation (A9)

def test_mixture_rate_reduces_to_single_tau():
    for tau in (0.55, 0.8, 1.0, 1.7):
        for rr, rb in ((1.0, 0.0), (0.3, 0.7), (0.0, 1.2)):
            assert math.isclose(O.omega(tau, tau, rr, rb), 1.0 / tau, rel_tol=1e-14)


def test_mixture_rate_harmonic_viscosity():
    # nu_bar from the density-weighted harmonic mean; nu = c_s^2 (1/omega - 1/2)
    tr, tb, rr, rb = 0.7, 1.3, 0.3, 0.9
    om = O.omega(tr, tb, rr, rb)
    nu = (1.0 / om - 0.5) / 3.0
    nu_r, nu_b = (tr - 0.5) / 3, (tb - 0.5) / 3
    x = rr / (rr + rb)
    assert math.isclose(1.0 / nu, x / nu_r + (1 - x) / nu_b, rel_tol=1e-13)


# ------------------------------------------------------------ EDM source (U3)

@pytest.mark.parametrize("omega", [0.0, 0.6, 1.25, 1.9])
def test_edm_source_moments(omega):
    c, w, _, _ = _tables()
    u = RNG.uniform(-0.05, 0.05, 3)
    du = RNG.uniform(-1e-3, 1e-3, 3)
    fk = O.feq(RNG.uniform(0.1, 1.5), RNG.uniform(-0.05, 0.05, 3)) + RNG.uniform(-1e-3, 1e-3, 19)
    rho_k = fk.sum()
    out = O.bgk_edm(omega, rho_k, u, du, fk)
    jk = fk @ c
    assert math.isclose(out.sum(), fk.sum(), rel_tol=1e-14)           # mass conserved
    assert np.allclose(out @ c, (1 - omega) * jk + omega * rho_k * u + rho_k * du,
                       atol=1e-15)                                      # momentum gets rho_k du
    # the source alone reproduces the shifted equilibrium's second moment change
    s = O.bgk_edm(0.0, rho_k, u, du, O.feq(rho_k, u)) - O.feq(rho_k, u)
    us = u + du
    assert np.allclose(np.einsum("i,ia,ib->ab", s, c, c),
                       rho_k * (np.outer(us, us) - np.outer(u, u)), atol=1e-15)


def test_bgk_relaxes_onto_equilibrium_at_unit_rate():
    rho, u = 0.8, np.array([0.02, -0.01, 0.03])
    fk = O.feq(rho, u)  # at equilibrium
    out = O.bgk_edm(1.0, rho, u, [0, 0, 0], RNG.uniform(0, 1, 19))
    assert np.allclose(out, O.feq(rho, u), atol=1e-16)
    assert np.allclose(O.bgk_edm(0.7, rho, u, [0, 0, 0], fk), fk, atol=1e-16)


# ---------------------------------------------------------- perturbation (U4)

@pytest.mark.parametrize("trial", range(6))
def test_perturbation_moments(trial):
    c, w, _, _ = _tables()
    A = RNG.uniform(0.001, 0.05)
    G = RNG.normal(size=3) * RNG.uniform(0.01, 0.5)
    g = np.linalg.norm(G)
    n = G / g
    p = O.perturbation(A, G)
    assert abs(p.sum()) < 1e-17
    assert np.allclose(p @ c, 0, atol=1e-17)
    m2 = np.einsum("i,ia,ib->ab", p, c, c)
    assert np.allclose(m2, -(A / 9.0) * g * (I3 - np.outer(n, n)), atol=1e-16)


def test_perturbation_vanishes_without_gradient():
    assert np.all(O.perturbation(0.01, [0, 0, 0]) == 0)
    assert np.all(O.perturbation(0.01, [1e-13, 0, 0], eps_g=1e-12) == 0)


# ----------------------------------------------------------- recolouring (U5)

@pytest.mark.parametrize("trial", range(6))
def test_recolouring_conserves_colour_and_splits_total(trial):
    c, w, _, _ = _tables()
    rr, rb = RNG.uniform(0.0, 1.0, 2)
    beta = RNG.uniform(0.3, 1.0)
    fstar = O.feq(rr + rb, RNG.uniform(-0.05, 0.05, 3)) + RNG.uniform(-1e-3, 1e-3, 19)
    fstar *= (rr + rb) / fstar.sum()
    G = RNG.normal(size=3)
    n = G / np.linalg.norm(G)
    outr, outb = O.recolour(rr, rb, fstar, G, beta)
    assert math.isclose(outr.sum(), rr, rel_tol=1e-13, abs_tol=1e-16)
    assert math.isclose(outb.sum(), rb, rel_tol=1e-13, abs_tol=1e-16)
    assert np.allclose(outr + outb, fstar, atol=1e-16)
    # colour flux: the proportional part plus 2 beta (rr rb / rho) sum_i w_i c_i c_i.n/|c_i|,
    # which is (1 + sqrt 2)/9 n for D3Q19
    rho = rr + rb
    flux = (outr - outb) @ c
    expect = ((rr - rb) / rho) * (fstar @ c) + 2 * beta * rr * rb / rho * (1 + math.sqrt(2)) / 9 * n
    assert np.allclose(flux, expect, atol=1e-15)


def test_recolouring_without_gradient_is_proportional():
    fstar = O.feq(1.0, [0.01, 0, 0])
    outr, outb = O.recolour(0.25, 0.75, fstar, [0, 0, 0], 0.7)
    assert np.allclose(outr, 0.25 * fstar, atol=1e-17)
    assert np.allclose(outb, 0.75 * fstar, atol=1e-17)


# ------------------------------------------------------ complete site update

@pytest.mark.parametrize("trial", range(4))
def test_site_collision_conservation(trial):
    c, w, _, _ = _tables()
    prm = O.Params(nx=1, ny=1, nz=1, tau_r=RNG.uniform(0.55, 1.5), tau_b=RNG.uniform(0.55, 1.5),
                   A=RNG.uniform(0, 0.02), beta=0.7)
    rr, rb = RNG.uniform(0.05, 1.0, 2)
    fr = O.feq(rr, RNG.uniform(-0.03, 0.03, 3)) + RNG.uniform(-1e-4, 1e-4, 19)
    fb = O.feq(rb, RNG.uniform(-0.03, 0.03, 3)) + RNG.uniform(-1e-4, 1e-4, 19)
    G = RNG.normal(size=3) * 0.3
    F = RNG.uniform(-1e-3, 1e-3, 3)
    outr, outb = O.collide_site(prm, fr, fb, G, F)
    assert math.isclose(outr.sum(), fr.sum(), rel_tol=1e-13)
    assert math.isclose(outb.sum(), fb.sum(), rel_tol=1e-13)
    assert np.allclose((outr + outb) @ c, (fr + fb) @ c + F, atol=1e-15)   # momentum + F


# ---------------------------------------------------- near-contact amplitude

def test_near_contact_amplitude_shape():
    A, hmin, K = 0.02, 3.0, 6
    assert O.nc_amplitude(A, hmin, K, 0) == 0.0
    for h in (1, 2, 3):
        assert O.nc_amplitude(A, hmin, K, h) == A            # constant up to h_min
    for h in (4, 5, 6):                                       # h^-3 beyond h_min
        assert math.isclose(O.nc_amplitude(A, hmin, K, h) * h ** 3, A * hmin ** 3, rel_tol=1e-14)
    assert O.nc_amplitude(A, hmin, K, K + 1) == 0.0          # out of probe range

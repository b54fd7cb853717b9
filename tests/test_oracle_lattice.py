"""Pins of the oracle's whole-lattice passes.

- streaming is an exact memory shift (Sec. 2, after eq:eq3): a bitwise
  permutation, equal to numpy.roll on periodic lattices, and time-reversible
  with halfway bounce-back walls;
- the colour-gradient stencil is exact on linear and quadratic phase fields and
  reads the mirror site at a halfway wall;
- rest states stay at rest; per-component mass and (unforced) momentum are
  conserved; a body force adds exactly F per site per step;
- the near-contact force on a one-dimensional film agrees with a brute-force
  scan of the rule written for that special case (Sec. 4, F_rep equation).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_12764_amd import workloads as W
from tests.helpers import oracle_params

C, Wt, OPP, _ = O.tables()


def _rand_pop(rng, shape):
    return rng.uniform(0.0, 1.0, size=(2, 19) + shape)


# ----------------------------------------------------------------- streaming (U7)

@pytest.mark.parametrize("n", [(1, 1, 1), (2, 3, 1), (4, 4, 4), (5, 3, 7)])
def test_periodic_streaming_is_roll(n):
    rng = np.random.default_rng(7)
    prm = O.Params(nx=n[0], ny=n[1], nz=n[2])
    fpost = _rand_pop(rng, prm.shape)
    f = O.stream(prm, fpost)
    for k in range(2):
        for i in range(19):
            cx, cy, cz = C[i]
            ref = np.roll(fpost[k, i], shift=(cz, cy, cx), axis=(0, 1, 2))
            assert np.array_equal(f[k, i], ref)


@pytest.mark.parametrize("bc", [(0, 1, 0), (1, 1, 1), (0, 1, 1), (1, 0, 0)])
@pytest.mark.parametrize("n", [(1, 1, 1), (3, 2, 4), (6, 5, 4)])
def test_wall_streaming_is_reversible_permutation(bc, n):
    rng = np.random.default_rng(11)
    prm = O.Params(nx=n[0], ny=n[1], nz=n[2], bc=bc)
    fpost = _rand_pop(rng, prm.shape)
    f = O.stream(prm, fpost)
    # a permutation: every value lands somewhere exactly once
    for k in range(2):
        assert np.array_equal(np.sort(f[k].ravel()), np.sort(fpost[k].ravel()))
    # reverse every direction, stream again, reverse: back to the start
    back = O.stream(prm, f[:, OPP])[:, OPP]
    assert np.array_equal(back, fpost)


def test_bounce_back_reflects_into_opposite_direction_at_the_source():
    prm = O.Params(nx=1, ny=1, nz=1, bc=(1, 1, 1))
    fpost = np.arange(38, dtype=np.float64).reshape(2, 19, 1, 1, 1)
    f = O.stream(prm, fpost)
    assert np.array_equal(f[:, OPP], fpost)


# ----------------------------------------------------------------- gradient (U6)

def test_gradient_exact_on_linear_and_quadratic_fields():
    n = 9
    prm = O.Params(nx=n, ny=n, nz=n)
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(np.float64)
    a = np.array([0.3, -0.2, 0.15])
    phi = 0.1 + a[0] * x + a[1] * y + a[2] * z + 0.02 * x * x - 0.03 * y * z
    G = O.phase_gradient(prm, phi)
    grad = np.stack([a[0] + 0.04 * x, a[1] - 0.03 * z, a[2] - 0.03 * y])
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))   # away from the wrap seam
    assert np.allclose(G[inner], grad[inner], atol=1e-14)


def test_gradient_uses_mirror_site_at_a_wall():
    ny = 6
    prm = O.Params(nx=3, ny=ny, nz=2, bc=(0, 1, 0))
    prof = np.array([0.9, 0.4, -0.1, -0.3, 0.2, 0.7])
    phi = np.broadcast_to(prof[None, :, None], prm.shape).copy()
    G = O.phase_gradient(prm, phi)
    ext = np.concatenate([[prof[0]], prof, [prof[-1]]])          # mirror across y=-1/2, ny-1/2
    expect = (ext[2:] - ext[:-2]) / 2.0
    assert np.allclose(G[1][0, :, 0], expect, atol=1e-15)
    assert np.allclose(G[0], 0, atol=1e-16) and np.allclose(G[2], 0, atol=1e-16)


# --------------------------------------------------------------- rest states (U8)

@pytest.mark.parametrize("red", [1.0, 0.0, 0.35])
def test_uniform_state_stays_uniform_and_at_rest(red):
    prm = O.Params(nx=4, ny=3, nz=5, tau_r=0.8, tau_b=1.1, A=0.01, beta=0.7,
                   nc_strength=0.02, nc_range=2)
    rr = np.full(prm.shape, red)
    rb = np.full(prm.shape, 1.0 - red)
    f0 = O.init(prm, rr, rb)
    f = O.step(prm, f0, 10)
    flat = f.reshape(2, 19, -1)
    assert np.all(flat == flat[:, :, :1])                 # translation invariant, bitwise
    _, _, j = O.moments(prm, f)
    assert np.all(j == 0.0)                               # no spurious momentum at all
    assert np.abs(f - f0).max() < 1e-15


# ------------------------------------------------------------- invariants (I2)

def test_mass_and_momentum_conservation_periodic():
    rng_shape = (6, 5, 7)
    rr, rb, u = W.random_state(3, rng_shape)
    prm = O.Params(nx=7, ny=5, nz=6, tau_r=0.7, tau_b=1.3, A=0.02, beta=0.7)
    f0 = O.init(prm, rr, rb, u)
    f = O.step(prm, f0, 20)
    r0, b0, j0 = O.moments(prm, f0)
    r1, b1, j1 = O.moments(prm, f)
    assert math.isclose(r1.sum(), r0.sum(), rel_tol=1e-13)
    assert math.isclose(b1.sum(), b0.sum(), rel_tol=1e-13)
    assert np.allclose(j1.sum(axis=(1, 2, 3)), j0.sum(axis=(1, 2, 3)), atol=1e-12)


def test_body_force_adds_exact_momentum():
    shape = (4, 5, 6)
    rr, rb, u = W.random_state(5, shape)
    F = np.array([1e-5, -2e-5, 3e-6])
    prm = O.Params(nx=6, ny=5, nz=4, tau_r=0.9, tau_b=0.9, A=0.01, beta=0.7,
                   body_force=tuple(F))
    f0 = O.init(prm, rr, rb, u)
    steps = 7
    f = O.step(prm, f0, steps)
    _, _, j0 = O.moments(prm, f0)
    _, _, j1 = O.moments(prm, f)
    N = rr.size
    assert np.allclose(j1.sum(axis=(1, 2, 3)) - j0.sum(axis=(1, 2, 3)), steps * N * F,
                       rtol=1e-9, atol=1e-13)


def test_mass_conservation_with_walls_and_near_contact():
    w = W.two_droplets(n=(40, 24, 6), R=6, gap=2.0, A=0.01, nc_strength=0.03, nc_range=2)
    p = dict(w.params)
    p["bc"] = (0, 1, 1)
    prm = oracle_params(p)
    f0 = O.init(prm, w.rho_r, w.rho_b)
    f = O.step(prm, f0, 30)
    r0, b0, _ = O.moments(prm, f0)
    r1, b1, _ = O.moments(prm, f)
    assert math.isclose(r1.sum(), r0.sum(), rel_tol=1e-13)
    assert math.isclose(b1.sum(), b0.sum(), rel_tol=1e-13)


# ------------------------------------------------------------ brute force (I7)

def test_moments_brute_force_4cubed():
    rng = np.random.default_rng(2)
    prm = O.Params(nx=4, ny=4, nz=4)
    f = _rand_pop(rng, prm.shape)
    rr, rb, j = O.moments(prm, f)
    for s in itertools.product(range(4), repeat=3):
        z, y, x = s
        assert math.isclose(rr[s], sum(f[0, i, z, y, x] for i in range(19)), rel_tol=1e-14)
        assert math.isclose(rb[s], sum(f[1, i, z, y, x] for i in range(19)), rel_tol=1e-14)
        for a in range(3):
            ref = sum((f[0, i, z, y, x] + f[1, i, z, y, x]) * C[i, a] for i in range(19))
            assert math.isclose(j[(a,) + s], ref, rel_tol=1e-12, abs_tol=1e-14)


# ----------------------------------------------------- near-contact on a film

def _film_force_brute(phi_line, strength, K, hmin, g_iface):
    """1-D special case: G = (phi(x+1) - phi(x-1))/2 (periodic), the outward
    normal is -sign(G), so the ray samples are x - k sign(G) exactly."""
    n = len(phi_line)
    G = np.array([(phi_line[(x + 1) % n] - phi_line[(x - 1) % n]) / 2 for x in range(n)])
    F = np.zeros(n)
    for x in range(n):
        if abs(G[x]) < g_iface:
            continue
        step = -1 if G[x] > 0 else 1
        for k in range(1, K + 1):
            y = (x + k * step) % n
            if abs(G[y]) >= g_iface and G[y] * G[x] < 0:
                amp = strength if k <= hmin else strength * (hmin / k) ** 3
                F[x] = amp * G[x]
                break
    return G, F


@pytest.mark.parametrize("K,hmin", [(2, 2.0), (4, 2.0), (3, 1.0)])
def test_near_contact_film_matches_brute_force(K, hmin):
    # two slabs of red separated by a thin blue film, along x
    n = 40
    x = np.arange(n, dtype=np.float64)
    phi = np.maximum(np.tanh((8 - np.abs(x - 10)) / 2), np.tanh((8 - np.abs(x - 29.5)) / 2))
    prm = O.Params(nx=n, ny=2, nz=3, nc_strength=0.02, nc_range=K, nc_hmin=hmin, eps_g=1e-12)
    field = np.broadcast_to(phi[None, None, :], prm.shape).copy()
    G = O.phase_gradient(prm, field)
    Fn = O.nearcontact(prm, G)
    Gb, Fb = _film_force_brute(phi, 0.02, K, hmin, 0.05)
    assert np.allclose(G[0, 1, 1], Gb, atol=1e-15)
    assert np.allclose(Fn[0, 1, 1], Fb, atol=1e-17)
    assert np.count_nonzero(Fb) > 0                                 # the film is detected
    assert np.abs(Fn[1]).max() < 1e-18 and np.abs(Fn[2]).max() < 1e-18    # round-off only
    assert np.all(Fb * Gb >= 0)                                     # points into its own slab


def test_near_contact_ignores_an_isolated_droplet():
    w = W.sphere(n=36, R=7.0)           # far from its own periodic images
    prm = oracle_params(dict(w.params, nc_strength=0.05, nc_range=3, nc_hmin=2.0))
    phi = (w.rho_r - w.rho_b) / (w.rho_r + w.rho_b)
    G = O.phase_gradient(prm, phi)
    assert np.all(O.nearcontact(prm, G) == 0.0)


def _diagonal_film_force_brute(phi_u, g_u, strength, K, hmin, g_iface):
    """Special case of a film whose phase field depends on u = a + b only (a, b
    two lattice axes, periodic, equal extents n): G lies along e_a + e_b, its
    two components equal (g_u at each u), so the outward normal is
    -sign(g_u)(e_a + e_b)/sqrt(2) and ray sample k sits at
    u - 2 round(k / sqrt 2) sign(g_u) (C rounding: halves away from zero)."""
    n = len(phi_u)
    gm = np.abs(g_u) * np.sqrt(2.0)           # |G| with two equal components
    F = np.zeros(n)
    for u in range(n):
        if gm[u] < g_iface:
            continue
        s = 1 if g_u[u] > 0 else -1
        for k in range(1, K + 1):
            off = int(np.floor(k / np.sqrt(2.0) + 0.5))
            v = (u - 2 * off * s) % n
            if gm[v] >= g_iface and g_u[v] * g_u[u] < 0:
                amp = strength if k <= hmin else strength * (hmin / k) ** 3
                F[u] = amp * g_u[u]
                break
    return F


@pytest.mark.parametrize("axes", [(2, 1), (2, 0), (1, 0)])
@pytest.mark.parametrize("K,hmin", [(2, 2.0), (4, 2.0)])
def test_near_contact_on_a_diagonal_film_matches_brute_force(axes, K, hmin):
    # two slabs of red and a thin blue film, constant along the lattice
    # diagonal of two axes: the probe's rays run along that diagonal, so its
    # sampling of off-axis normals (the rounding of k n in two components at
    # once) reduces to a scan in u = a + b
    n = 24
    a, b = axes                                     # array axes (z = 0, y = 1, x = 2)
    shape = [3, 3, 3]
    shape[a] = shape[b] = n
    u = np.arange(n, dtype=np.float64)
    phi_u = np.maximum(np.tanh((5 - np.abs(u - 6)) / 2), np.tanh((5 - np.abs(u - 18.5)) / 2))
    idx = np.indices(shape)
    field = phi_u[(idx[a] + idx[b]) % n]
    prm = O.Params(nx=shape[2], ny=shape[1], nz=shape[0], nc_strength=0.02, nc_range=K, nc_hmin=hmin,
                   eps_g=1e-12)
    G = O.phase_gradient(prm, field)
    comp = {2: 0, 1: 1, 0: 2}                       # array axis -> component of G (x, y, z)
    ga, gb = G[comp[a]], G[comp[b]]
    assert np.allclose(ga, gb, atol=1e-15)          # G along the diagonal
    other = 3 - comp[a] - comp[b]
    assert np.abs(G[other]).max() < 1e-15
    sel = [1, 1, 1]
    sel[b] = 0                                      # the line a + 0 runs through every u
    line = tuple(slice(None) if k == a else sel[k] for k in range(3))
    g_u = ga[line]
    Fn = O.nearcontact(prm, G)
    Fb = _diagonal_film_force_brute(phi_u, g_u, 0.02, K, hmin, 0.05)
    assert np.count_nonzero(Fb) > 0                 # the film is detected
    assert np.allclose(Fn[comp[a]][line], Fb, atol=1e-17)
    assert np.allclose(Fn[comp[b]][line], Fb, atol=1e-17)
    assert np.abs(Fn[other]).max() < 1e-18


@pytest.mark.parametrize("K,hmin", [(2, 2.0), (4, 2.0)])
def test_near_contact_on_a_body_diagonal_film_matches_brute_force(K, hmin):
    # the same along the body diagonal: phi depends on u = x + y + z, G has
    # three equal components, ray sample k sits at u - 3 round(k / sqrt 3) sign
    n = 24
    u = np.arange(n, dtype=np.float64)
    phi_u = np.maximum(np.tanh((5 - np.abs(u - 6)) / 2), np.tanh((5 - np.abs(u - 18.5)) / 2))
    z, y, x = np.indices((n, n, n))
    field = phi_u[(x + y + z) % n]
    prm = O.Params(nx=n, ny=n, nz=n, nc_strength=0.02, nc_range=K, nc_hmin=hmin, eps_g=1e-12)
    G = O.phase_gradient(prm, field)
    assert np.allclose(G[0], G[1], atol=1e-15) and np.allclose(G[0], G[2], atol=1e-15)
    g_u = G[0][0, 0, :]                             # the line y = z = 0 runs through every u
    gm = np.abs(g_u) * np.sqrt(3.0)
    Fb = np.zeros(n)
    for k0 in range(n):
        if gm[k0] < 0.05:
            continue
        s = 1 if g_u[k0] > 0 else -1
        for k in range(1, K + 1):
            v = (k0 - 3 * int(np.floor(k / np.sqrt(3.0) + 0.5)) * s) % n
            if gm[v] >= 0.05 and g_u[v] * g_u[k0] < 0:
                Fb[k0] = (0.02 if k <= hmin else 0.02 * (hmin / k) ** 3) * g_u[k0]
                break
    Fn = O.nearcontact(prm, G)
    assert np.count_nonzero(Fb) > 0
    for c in range(3):
        assert np.allclose(Fn[c][0, 0, :], Fb, atol=1e-17)

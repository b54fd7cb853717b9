"""Pins of the oracle's Shan-Chen interface model (Sec. 2.1, eq. shanchen_force
entering eq:edm), independent of the oracle's own code: closed forms of the
D3Q19 stencil on trigonometric fields, exact conservation identities, the
mirror rule at walls, the sign of G_C through the physics (G_C > 0 separates a
mixture, G_C < 0 does not), and Laplace's law for discs."""
import numpy as np
import pytest

from oracle import oracle as O


def sc_params(n, **kw):
    nz = kw.pop("nz", n)
    ny = kw.pop("ny", n)
    return O.Params(nx=n, ny=ny, nz=nz, model=1, **kw)


def test_force_on_axis_sinusoids_matches_closed_form():
    # rho_b = 1 + e sin(k v) along one axis v: the stencil sum over the five
    # directions with c_v = +1 (weights 1/18 + 4/36 = 1/6) minus those with
    # c_v = -1 gives (1/6)(rho(v+1) - rho(v-1)) = (e/3) sin(k) cos(k v), so
    # F^r_v = -G rho_r (e/3) sin(k) cos(k v) and the other components vanish.
    n, e, G = 12, 0.1, 1.7
    k = 2 * np.pi / n
    prm = sc_params(n, g_sc=G)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for axis, v in enumerate((x, y, z)):
        rb = 1.0 + e * np.sin(k * v)
        rr = np.full_like(rb, 0.3)
        Fr, Fb = O.sc_force(prm, rr, rb)
        want = -G * 0.3 * (e / 3.0) * np.sin(k) * np.cos(k * v)
        for a in range(3):
            np.testing.assert_allclose(Fr[a], want if a == axis else 0.0, atol=1e-15)
        # rho_r is uniform: the force on the blue component vanishes
        np.testing.assert_allclose(Fb, 0.0, atol=1e-15)


def test_force_on_product_sinusoid_involves_the_diagonal_weights():
    # rho_b = 1 + e sin(a x) sin(b y): the x-sum collects
    # [sin(a(x+1)) - sin(a(x-1))] sin(b y) [w1 + 2 w2 (1 + cos b)]
    # = (1/9) sin(a) cos(a x) sin(b y) (2 + cos b) with w1 = 1/18, w2 = 1/36.
    n, e, G = 12, 0.05, 2.0
    a = 2 * np.pi / n
    b = 4 * np.pi / n
    prm = sc_params(n, g_sc=G)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    rb = 1.0 + e * np.sin(a * x) * np.sin(b * y)
    rr = np.full_like(rb, 0.5)
    Fr, _ = O.sc_force(prm, rr, rb)
    sx = e * np.sin(a) * np.cos(a * x) * np.sin(b * y) * (2 + np.cos(b)) / 9.0
    sy = e * np.sin(b) * np.cos(b * y) * np.sin(a * x) * (2 + np.cos(a)) / 9.0
    np.testing.assert_allclose(Fr[0], -G * 0.5 * sx, atol=1e-15)
    np.testing.assert_allclose(Fr[1], -G * 0.5 * sy, atol=1e-15)
    np.testing.assert_allclose(Fr[2], 0.0, atol=1e-15)


def test_total_force_vanishes_on_a_periodic_lattice():
    # sum_x rho_r(x) sum_i w_i rho_b(x+c_i) c_i + sum_x rho_b(x) sum_i w_i
    # rho_r(x+c_i) c_i = 0: shifting x -> x - c_i in the second sum and
    # pairing c_i with -c_i turns it into minus the first.
    rng = np.random.default_rng(3)
    prm = sc_params(7, ny=5, nz=6, g_sc=2.3)
    rr = rng.uniform(0.1, 1.0, prm.shape)
    rb = rng.uniform(0.1, 1.0, prm.shape)
    Fr, Fb = O.sc_force(prm, rr, rb)
    tot = (Fr + Fb).reshape(3, -1).sum(1)
    scale = np.abs(Fr).sum()
    assert np.all(np.abs(tot) <= 1e-14 * scale), tot
    # ... and does not vanish for each component alone
    assert np.abs(Fr.reshape(3, -1).sum(1)).max() > 1e-3 * scale / rr.size


def test_mirror_rule_at_walls():
    # walls in y: a field depending on y only; at y = 0 the neighbour y = -1
    # is the mirror image y = 0, so the y-sum is (1/6)(rho(1) - rho(0)); at
    # y = n-1 it is (1/6)(rho(n-1) - rho(n-2)); inside (1/6)(rho(y+1) - rho(y-1)).
    n, G = 6, 1.3
    prm = sc_params(4, ny=n, nz=3, bc=(0, 1, 0), g_sc=G)
    prof = np.array([0.2, 0.5, 0.9, 0.4, 0.7, 0.1])
    rb = np.broadcast_to(prof[None, :, None], prm.shape).copy()
    rr = np.ones(prm.shape)
    Fr, _ = O.sc_force(prm, rr, rb)
    ext = np.concatenate([[prof[0]], prof, [prof[-1]]])
    want = -G * (ext[2:] - ext[:-2]) / 6.0
    np.testing.assert_allclose(Fr[1][0, :, 0], want, atol=1e-15)
    np.testing.assert_allclose(Fr[0], 0.0, atol=1e-15)
    np.testing.assert_allclose(Fr[2], 0.0, atol=1e-15)


def test_site_collision_conserves_mass_and_adds_the_force():
    # BGK toward f^eq(rho_k, u) with the common u = j/rho conserves each
    # component's mass and the total momentum; each exact-difference source
    # adds rho_k du_k = F^k (Sec. 2.1): component momentum
    # j_k' = (1 - w) j_k + w rho_k u + F^k with F^k = F^k_SC + (rho_k/rho) F_body.
    rng = np.random.default_rng(5)
    c, w, _, _ = O.tables()
    prm = sc_params(4, g_sc=1.9, tau_r=0.8, tau_b=1.3, body_force=(1e-3, -2e-3, 5e-4))
    fr = w * 0.6 * (1 + rng.uniform(-0.2, 0.2, 19))
    fb = w * 0.4 * (1 + rng.uniform(-0.2, 0.2, 19))
    Fr = np.array([0.01, -0.02, 0.005])
    Fb = np.array([-0.007, 0.013, 0.002])
    outr, outb = O.sc_collide_site(prm, fr, fb, Fr, Fb)
    assert abs(outr.sum() - fr.sum()) <= 1e-15
    assert abs(outb.sum() - fb.sum()) <= 1e-15
    rr, rb = fr.sum(), fb.sum()
    rho = rr + rb
    u = (fr + fb) @ c / rho
    om = O.omega(0.8, 1.3, rr, rb)
    F = np.array(prm.body_force)
    for f, out, Fk, rk in ((fr, outr, Fr, rr), (fb, outb, Fb, rb)):
        want = (1 - om) * (f @ c) + om * rk * u + Fk + (rk / rho) * F
        np.testing.assert_allclose(out @ c, want, atol=1e-15)


def test_uniform_mixture_is_a_fixed_point():
    prm = sc_params(6, g_sc=3.0)
    rr = np.full(prm.shape, 0.5)
    rb = np.full(prm.shape, 0.5)
    f = O.init(prm, rr, rb)
    g = O.step(prm, f, 5)
    # every site stays identical (bitwise), at the equilibrium up to rounding
    np.testing.assert_array_equal(g, np.broadcast_to(g[..., :1, :1, :1], g.shape))
    np.testing.assert_allclose(g, f, atol=1e-16)


def _separation(G, n=16, steps=300, seed=0):
    rng = np.random.default_rng(seed)
    prm = sc_params(n, g_sc=G)
    phi0 = rng.uniform(-0.01, 0.01, prm.shape)
    f = O.init(prm, 0.5 * (1 + phi0), 0.5 * (1 - phi0))
    f = O.step(prm, f, steps)
    rr, rb, _ = O.moments(prm, f)
    return float(((rr - rb) / (rr + rb)).std()), float(phi0.std())


def test_positive_coupling_separates_and_negative_mixes():
    # The paper: G_C > 0 is repulsive.  A symmetric mixture of total density 1
    # demixes for large enough repulsion and stays mixed otherwise.
    sep, s0 = _separation(3.0)
    assert sep > 0.5, sep
    for G in (0.5, -1.5):
        s, s0 = _separation(G)
        assert s < s0, (G, s, s0)


def _disc_jump(G, R, n=64, steps=3000):
    prm = sc_params(n, nz=1, g_sc=G)
    y, x = np.mgrid[0:n, 0:n]
    r = np.sqrt((x - (n - 1) / 2) ** 2 + (y - (n - 1) / 2) ** 2)
    phi0 = np.tanh((R - r) / 2.0)[None]
    f = O.init(prm, 0.5 * (1 + phi0), 0.5 * (1 - phi0))
    f = O.step(prm, f, steps)
    rr, rb, _ = O.moments(prm, f)
    # bulk pressure of the model: c_s^2 rho + G c_s^2 rho_r rho_b
    p = ((rr + rb) / 3.0 + G / 3.0 * rr * rb)[0]
    Rm = np.sqrt((rr[0] > rb[0]).sum() / np.pi)
    return Rm, p[r < Rm - 4].mean() - p[r > Rm + 4].mean()


@pytest.mark.slow
def test_laplace_law_for_discs():
    # 2-D discs: the pressure jump is sigma/R, so dp * R is the same for every
    # radius (measured radius from the area of the red phase).
    prods = []
    for R in (8.0, 12.0, 16.0):
        Rm, dp = _disc_jump(2.5, R)
        assert dp > 0
        prods.append(dp * Rm)
    prods = np.array(prods)
    assert prods.max() / prods.min() < 1.04, prods

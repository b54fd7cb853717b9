"""Pins of the oracle's Korteweg-tensor diagnostic (Sec. 4.1: the Korteweg
tensor from the Laplacian and the gradient products of the field, and the
projection of fine data by block averages).

The D3Q19 stencils have closed forms on trigonometric fields, worked out by
hand from the lattice weights (1/3 rest, 1/18 axis, 1/36 face diagonal):
for phi = sin(kx x) sin(ky y) on a periodic lattice

    d_x phi = sin(kx) cos(kx x) sin(ky y) (2 + cos ky) / 3
    d_y phi = sin(ky) sin(kx x) cos(ky y) (2 + cos kx) / 3
    Lap phi = phi [ (2/3)(2 cos kx + 2 cos ky + cos kx cos ky + 1) - 4 ]

(the diagonal directions supply the cos ky and cos kx cos ky terms, so a
dropped diagonal, a wrong weight or a wrong sign fails them), and for a field
of x alone next to halfway walls the mirror rule gives
d_x phi = (phi(x+1) - phi(x-1))/2 and Lap phi = phi(x+1) + phi(x-1) - 2 phi(x)
with phi(-1) = phi(0), phi(n) = phi(n-1).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _prm(nx, ny, nz, bc=(0, 0, 0)):
    return O.Params(nx=nx, ny=ny, nz=nz, bc=bc, tau_r=1.0, tau_b=1.0, A=0.0, beta=0.7)


def _grid(prm):
    z, y, x = np.meshgrid(np.arange(prm.nz), np.arange(prm.ny), np.arange(prm.nx), indexing="ij")
    return x.astype(float), y.astype(float), z.astype(float)


def test_product_wave_matches_closed_forms():
    prm = _prm(24, 16, 3)
    x, y, _ = _grid(prm)
    kx, ky = 2 * math.pi * 2 / 24, 2 * math.pi / 16
    phi = np.sin(kx * x) * np.sin(ky * y)
    lam = 0.37
    K = O.korteweg(prm, phi, lam)
    gx = math.sin(kx) * np.cos(kx * x) * np.sin(ky * y) * (2 + math.cos(ky)) / 3
    gy = math.sin(ky) * np.sin(kx * x) * np.cos(ky * y) * (2 + math.cos(kx)) / 3
    lap = phi * ((2 / 3) * (2 * math.cos(kx) + 2 * math.cos(ky) + math.cos(kx) * math.cos(ky) + 1) - 4)
    # off-diagonals are the gradient products alone
    assert np.abs(K[3] + lam * gx * gy).max() < 1e-15
    assert np.abs(K[4]).max() < 1e-15 and np.abs(K[5]).max() < 1e-15
    # K_zz has no gradient product: lam (phi Lap + |grad|^2 / 2)
    iso = lam * (phi * lap + 0.5 * (gx * gx + gy * gy))
    assert np.abs(K[2] - iso).max() < 1e-15
    # the diagonal differences are the squared derivatives
    assert np.abs((K[2] - K[0]) - lam * gx * gx).max() < 1e-15
    assert np.abs((K[2] - K[1]) - lam * gy * gy).max() < 1e-15


def test_continuum_limit_of_a_long_wave():
    # k -> 0: the stencils tend to the derivatives with relative errors
    # -k^2/6 (gradient) and -k^2/12 (Laplacian), so K_xx, itself O(k^2),
    # is off by O(k^4); a first-order stencil would be off by O(k^3)
    prm = _prm(256, 4, 2)
    x, _, _ = _grid(prm)
    k = 2 * math.pi / 256
    phi = np.cos(k * x)
    K = O.korteweg(prm, phi, 1.0)
    gx = -k * np.sin(k * x)
    lap = -k * k * phi
    ref_xx = phi * lap + 0.5 * gx * gx - gx * gx
    err = np.abs(K[0] - ref_xx).max()
    assert err < 0.25 * k ** 4 and err > 0.01 * k ** 4


def test_mirror_rule_at_walls():
    prm = _prm(8, 3, 2, bc=(1, 0, 0))
    x, _, _ = _grid(prm)
    phi = x.copy()
    K = O.korteweg(prm, phi, 1.0)
    gx = np.where((x == 0) | (x == 7), 0.5, 1.0)
    lap = np.where(x == 0, 1.0, np.where(x == 7, -1.0, 0.0))
    # 1-D field: K_yy = K_zz = phi Lap + gx^2/2, K_xx = that - gx^2
    assert np.abs(K[1] - (phi * lap + 0.5 * gx * gx)).max() < 1e-14
    assert np.abs(K[2] - K[1]).max() == 0.0
    assert np.abs(K[1] - K[0] - gx * gx).max() < 1e-14


def test_constant_field_is_stress_free_and_lambda_is_linear():
    prm = _prm(6, 5, 4, bc=(0, 1, 1))
    assert np.abs(O.korteweg(prm, np.full(prm.shape, 0.3), 2.0)).max() == 0.0
    rng = np.random.default_rng(3)
    phi = rng.uniform(-1, 1, prm.shape)
    K1 = O.korteweg(prm, phi, 1.0)
    K3 = O.korteweg(prm, phi, 3.0)
    assert np.abs(K3 - 3.0 * K1).max() < 1e-14


def test_block_average_projection():
    prm = _prm(8, 4, 12)
    rng = np.random.default_rng(5)
    # a field constant on each 4-block averages to that constant
    blocks = rng.uniform(-1, 1, (3, 1, 2))
    field = np.kron(blocks, np.ones((4, 4, 4)))
    assert np.abs(O.block_average(prm, field, 4) - blocks).max() < 1e-15
    # the mean of the block means is the mean of the field; b = 1 is the identity
    f = rng.normal(size=(2,) + prm.shape)
    for b in (1, 2, 4):
        c = O.block_average(prm, f, b)
        assert c.shape == (2, 12 // b, 4 // b, 8 // b)
        assert np.abs(c.mean(axis=(1, 2, 3)) - f.mean(axis=(1, 2, 3))).max() < 1e-15
    assert np.array_equal(O.block_average(prm, f, 1), f)
    with pytest.raises(ValueError):
        O.block_average(prm, f, 3)


def test_phase_field_of_an_initial_state():
    prm = _prm(5, 4, 3)
    rng = np.random.default_rng(1)
    rr = rng.uniform(0.1, 1.0, prm.shape)
    rb = rng.uniform(0.1, 1.0, prm.shape)
    f = O.init(prm, rr, rb)
    assert np.abs(O.phase_field(prm, f) - (rr - rb) / (rr + rb)).max() < 1e-15

"""Shared test helpers: parameter conversion and the parity metrics."""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

def oracle_params(p: dict, eps_g=None, g_iface=0.05) -> O.Params:
    """Oracle parameters for a library parameter dict (same quantities)."""
    return O.params_from_dict(p, eps_g=eps_g, g_iface=g_iface)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def state_errors(f, f_ref):
    """Parity metric: the largest relative L2 error over the 38 population
    fields and the two component densities; momentum is measured against
    c_s * ||rho_ref|| because the reference momentum itself is tiny."""
    errs = {}
    worst = 0.0
    for k in range(2):
        for i in range(19):
            e = rel_l2(f[k, i], f_ref[k, i])
            worst = max(worst, e)
    errs["populations"] = worst
    rr, rb = f[0].sum(0), f[1].sum(0)
    rr0, rb0 = f_ref[0].sum(0), f_ref[1].sum(0)
    errs["rho_r"] = rel_l2(rr, rr0)
    errs["rho_b"] = rel_l2(rb, rb0)
    c, _, _, _ = O.tables()
    j = np.einsum("kixyz,ia->axyz", f, c.astype(np.float64))
    j0 = np.einsum("kixyz,ia->axyz", f_ref, c.astype(np.float64))
    rho0 = rr0 + rb0
    errs["momentum"] = float(np.linalg.norm((j - j0).ravel()) /
                             (np.sqrt(1.0 / 3.0) * np.linalg.norm(rho0.ravel())))
    errs["max_abs"] = float(np.abs(f - f_ref).max())
    errs["worst"] = max(errs["populations"], errs["rho_r"], errs["rho_b"], errs["momentum"])
    return errs


def duct_series(a, b, y, z, g, nu, nmax=199):
    """Steady duct flow u(y, z) for a width a (y in [-a/2, a/2]) by height b
    (z in [-b/2, b/2]) cross-section under force density g: the plane profile
    (g / 2 nu)(a^2/4 - y^2), expanded in cos(n pi y / a) over odd n, corrected
    by the cosh(n pi z / a) terms that vanish at z = +-b/2."""
    u = np.zeros(np.broadcast(y, z).shape)
    for n in range(1, nmax + 1, 2):
        u += ((-1) ** ((n - 1) // 2) / n ** 3
              * (1 - np.cosh(n * math.pi * z / a) / np.cosh(n * math.pi * b / (2 * a)))
              * np.cos(n * math.pi * y / a))
    return 4 * g * a * a / (nu * math.pi ** 3) * u


def structure_factor(phi):
    """Shell-averaged |FFT(phi - <phi>)|^2 of a cubic field: the first
    moment k1 = sum k S / sum S and the peak height (k in units of 2 pi / n)."""
    n = phi.shape[0]
    f = np.fft.fftn(phi - phi.mean())
    p = (f.real ** 2 + f.imag ** 2).ravel()
    k1d = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1d, k1d, k1d, indexing="ij")
    kk = np.rint(np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)).astype(int).ravel()
    m = kk <= n // 2
    S = np.bincount(kk[m], weights=p[m], minlength=n // 2 + 1)
    cnt = np.bincount(kk[m], minlength=n // 2 + 1)
    S = S / np.maximum(cnt, 1)
    k = np.arange(n // 2 + 1)
    return float((k[1:] * S[1:]).sum() / S[1:].sum()), float(S[1:].max())

"""Shared test helpers: parameter conversion and the parity metrics."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

EPS_G = {0: 1e-12, 1: 1e-6, 2: 1e-6, 3: 1e-6}


def oracle_params(p: dict, eps_g=None, g_iface=0.05) -> O.Params:
    """Oracle parameters for a library parameter dict (same quantities)."""
    if eps_g is None:
        eps_g = EPS_G[int(p.get("storage", 0))]
    return O.Params(nx=p["nx"], ny=p["ny"], nz=p["nz"], bc=tuple(p["bc"]),
                    tau_r=p["tau_r"], tau_b=p["tau_b"], A=p["A"], beta=p["beta"],
                    nc_strength=p["nc_strength"], nc_range=p["nc_range"],
                    nc_hmin=p["nc_hmin"], body_force=tuple(p["body_force"]),
                    eps_g=eps_g, g_iface=g_iface,
                    wall_velocity=tuple(map(tuple, p.get("wall_velocity", ((0.0, 0.0, 0.0),) * 6))),
                    model=int(p.get("model", 0)), g_sc=float(p.get("g_sc", 0.0)))


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

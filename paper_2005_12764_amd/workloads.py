"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds initial fields and parameter sets.  It contains none of
the update's arithmetic, so both the GPU path and the FP64 oracle consume
exactly the same arrays.  Every generator is deterministic in its seed
(``numpy.random.default_rng``).

Initial state convention: a phase field phi0 in [-1, 1] (+1 red / dispersed,
-1 blue / continuous) and a total density rho0, turned into component densities
rho_r = rho0 (1 + phi0) / 2 and rho_b = rho0 (1 - phi0) / 2.  A droplet of
radius R is phi0 = tanh((R - r) / 2) (a tanh interface of width 2); several
droplets take the maximum over droplets, with periodic minimum-image distances
on periodic axes.

The paper's applications (Sec. 4 microfluidic crystals, Sec. 5 bijels) are
simulation set-ups, not datasets: the functions below stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Storage codes of the library's parameter block.
F64, F32, F16, BF16 = 0, 1, 2, 3


@dataclass
class Workload:
    """Initial fields plus the lattice parameters of one run."""
    name: str
    params: dict
    rho_r: np.ndarray            # (nz, ny, nx) float64
    rho_b: np.ndarray
    u: Optional[np.ndarray] = None   # (3, nz, ny, nx) or None
    steps: int = 0
    info: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.rho_r.shape

    @property
    def sites(self) -> int:
        return int(self.rho_r.size)


def base_params(nx, ny, nz, **kw) -> dict:
    p = dict(nx=nx, ny=ny, nz=nz, bc=(0, 0, 0), storage=F32, tau_r=1.0, tau_b=1.0,
             A=0.0, beta=0.7, nc_strength=0.0, nc_range=0, nc_hmin=2.0,
             body_force=(0.0, 0.0, 0.0))
    p.update(kw)
    return p


def split_components(phi0: np.ndarray, rho0) -> tuple:
    rho0 = np.broadcast_to(np.asarray(rho0, dtype=np.float64), phi0.shape)
    return rho0 * (1.0 + phi0) / 2.0, rho0 * (1.0 - phi0) / 2.0


def _axis_dist(coord: np.ndarray, c: float, n: int, periodic: bool) -> np.ndarray:
    d = coord - c
    if periodic:
        d = d - n * np.round(d / n)
    return d


def droplet_phase(shape, centres, radii, bc=(0, 0, 0), width: float = 2.0,
                  background: float = -1.0) -> np.ndarray:
    """phi0 = max(background, max_j tanh((R_j - d_j)/width)) over droplets
    with d_j <= R_j + 6 width (the library's droplet initialiser uses the same
    rule); only a box around each droplet is touched, so many droplets on a
    big lattice stay cheap."""
    nz, ny, nx = shape
    n = (nx, ny, nz)
    phi = np.full(shape, background, dtype=np.float64)
    for c, R in zip(centres, radii):
        reach = int(math.ceil(R + 6 * width))
        idx = []
        dist = []
        for a in range(3):
            periodic = bc[a] == 0
            lo, hi = int(math.floor(c[a] - reach)), int(math.ceil(c[a] + reach))
            if periodic and hi - lo + 1 >= n[a]:
                lo, hi = 0, n[a] - 1
            coords = np.arange(lo, hi + 1)
            if periodic:
                coords = np.unique(np.mod(coords, n[a]))
            else:
                coords = coords[(coords >= 0) & (coords < n[a])]
            idx.append(coords)
            dist.append(_axis_dist(coords.astype(np.float64), c[a], n[a], periodic))
        if any(len(ix) == 0 for ix in idx):
            continue
        dx, dy, dz = dist
        r = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
        val = np.where(r <= R + 6 * width, np.tanh((R - r) / width), background)
        sub = np.ix_(idx[2], idx[1], idx[0])
        phi[sub] = np.maximum(phi[sub], val)
    return phi


def rsa_place(rng, n, radii, gap=1.0, bc=(0, 0, 0), attempts=10**6, batch=512):
    """Random sequential addition, largest droplet first: each centre is drawn
    uniformly until d_ij >= R_i + R_j + gap holds against every placed droplet
    (periodic minimum image on periodic axes, walls keep R + gap clear).
    Returns the placed centres and radii (droplets that found no room within
    ``attempts`` draws are dropped)."""
    order = np.argsort(-np.asarray(radii), kind="stable")
    radii = np.asarray(radii, dtype=np.float64)[order]
    n = np.asarray(n, dtype=np.float64)
    per = np.array([b == 0 for b in bc])
    placed_c = np.zeros((0, 3))
    placed_r = np.zeros(0)
    for R in radii:
        lo = np.where(per, 0.0, R + gap - 0.5)
        hi = np.where(per, n, n - 1 - (R + gap - 0.5))
        if np.any(hi <= lo):
            continue
        done = False
        tried = 0
        while tried < attempts and not done:
            cand = lo + rng.random((batch, 3)) * (hi - lo)
            tried += batch
            if len(placed_r) == 0:
                ok = np.ones(batch, dtype=bool)
            else:
                d = cand[:, None, :] - placed_c[None, :, :]
                d = np.where(per, d - n * np.round(d / n), d)
                dist = np.sqrt((d ** 2).sum(-1))
                ok = np.all(dist >= R + placed_r[None, :] + gap, axis=1)
            if ok.any():
                k = int(np.argmax(ok))
                placed_c = np.vstack([placed_c, cand[k]])
                placed_r = np.append(placed_r, R)
                done = True
    return placed_c, placed_r


def emulsion(rng, n, phi_v, rmin, rmax, bc=(0, 0, 0), gap=1.0, attempts=10**6):
    """Random emulsion of non-overlapping droplets at volume fraction phi_v.
    Radii are U[rmin, rmax]; droplets are drawn until their volume reaches
    phi_v of the box, then placed by RSA.  If RSA cannot reach the target
    (beyond its jamming limit), all radii are inflated uniformly by
    (target/achieved)^(1/3) and allowed to overlap (they merge)."""
    V = float(n[0] * n[1] * n[2])
    radii = []
    vol = 0.0
    while vol < phi_v * V:
        R = rng.uniform(rmin, rmax)
        radii.append(R)
        vol += 4.0 / 3.0 * math.pi * R ** 3
    centres, placed = rsa_place(rng, n, radii, gap=gap, bc=bc, attempts=attempts)
    achieved = float((4.0 / 3.0 * math.pi * placed ** 3).sum() / V)
    inflate = 1.0
    if achieved < 0.98 * phi_v and achieved > 0:
        inflate = (phi_v / achieved) ** (1.0 / 3.0)
        placed = placed * inflate
    return centres, placed, dict(target_phi_v=phi_v, rsa_phi_v=achieved, inflate=inflate,
                                 n_droplets=int(len(placed)))


# ---------------------------------------------------------------------------
# The five benchmark set-ups
# ---------------------------------------------------------------------------

def single_droplet(seed=0, n=32, R=8.0, storage=F64, tau=1.0, A=0.01, beta=0.7,
                   noise=1e-4, steps=200) -> Workload:
    """32^3 periodic box, one droplet of radius 8 centred at ((n-1)/2,)*3 so
    the set-up is mirror symmetric, density noise U(-noise, noise)."""
    rng = np.random.default_rng(seed)
    c = (n - 1) / 2.0
    phi0 = droplet_phase((n, n, n), [(c, c, c)], [R])
    rho0 = 1.0 + rng.uniform(-noise, noise, size=(n, n, n))
    rr, rb = split_components(phi0, rho0)
    p = base_params(n, n, n, storage=storage, tau_r=tau, tau_b=tau, A=A, beta=beta)
    return Workload("single_droplet_%d^3_R%g" % (n, R), p, rr, rb, None, steps,
                    dict(seed=seed, R=R))


def periodic_emulsion(seed=0, n=256, phi_v=0.30, rmin=6.0, rmax=12.0, storage=F32, tau=0.8,
                      A=0.005, beta=0.7, nc_strength=0.02, nc_range=2, steps=1000) -> Workload:
    """n^3 periodic emulsion: radii U[rmin, rmax], RSA to phi_v, near-contact
    repulsion of the given strength over nc_range sites (h_min = range)."""
    rng = np.random.default_rng(seed)
    cen, rad, info = emulsion(rng, (n, n, n), phi_v, rmin, rmax)
    phi0 = droplet_phase((n, n, n), cen, rad)
    rr, rb = split_components(phi0, 1.0)
    p = base_params(n, n, n, storage=storage, tau_r=tau, tau_b=tau, A=A, beta=beta,
                    nc_strength=nc_strength, nc_range=nc_range, nc_hmin=float(nc_range))
    info.update(seed=seed)
    return Workload("emulsion_%d^3_phi%.2f" % (n, phi_v), p, rr, rb, None, steps, info)


def crystal_channel(seed=0, nx=512, ny=128, nz=64, R=10.0, spacing=22.0, storage=F32, tau=0.7,
                    A=0.005, beta=0.7, nc_strength=0.02, nc_range=2, force=1e-6,
                    steps=2000) -> Workload:
    """Microfluidic-crystal channel: walls at y and z, periodic x, body force
    along x.  One hexagonal layer of droplets at mid-height: rows along x at
    x = spacing/2 + spacing*j, six rows at y = ny/2 - 1/2 + (m - 2.5) *
    spacing*sqrt(3)/2, odd rows shifted by spacing/2, integer jitter in
    {-1, 0, 1} per axis."""
    rng = np.random.default_rng(seed)
    per_row = int((nx - spacing / 2) // spacing) + 1
    rows = 6
    cen = []
    for m in range(rows):
        y = (ny - 1) / 2.0 + (m - (rows - 1) / 2.0) * spacing * math.sqrt(3) / 2.0
        for j in range(per_row):
            x = spacing / 2.0 + spacing * j + (spacing / 2.0 if m % 2 else 0.0)
            jit = rng.integers(-1, 2, size=3)
            cen.append((x + jit[0], y + jit[1], (nz - 1) / 2.0 + jit[2]))
    cen = [c for c in cen if c[0] < nx]
    phi0 = droplet_phase((nz, ny, nx), cen, [R] * len(cen), bc=(0, 1, 1))
    rr, rb = split_components(phi0, 1.0)
    p = base_params(nx, ny, nz, bc=(0, 1, 1), storage=storage, tau_r=tau, tau_b=tau, A=A,
                    beta=beta, nc_strength=nc_strength, nc_range=nc_range,
                    nc_hmin=float(nc_range), body_force=(force, 0.0, 0.0))
    return Workload("crystal_channel_%dx%dx%d" % (nx, ny, nz), p, rr, rb, None, steps,
                    dict(seed=seed, n_droplets=len(cen)))


def spinodal(seed=0, n=384, amp=0.01, storage=F32, tau=1.0, A=0.01, beta=0.7,
             nc_strength=0.03, nc_range=2, steps=5000) -> Workload:
    """Symmetric 50/50 mixture with phase noise U(-amp, amp), rho0 = 1."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(-amp, amp, size=(n, n, n))
    rr, rb = split_components(phi0, 1.0)
    p = base_params(n, n, n, storage=storage, tau_r=tau, tau_b=tau, A=A, beta=beta,
                    nc_strength=nc_strength, nc_range=nc_range, nc_hmin=float(nc_range))
    return Workload("spinodal_%d^3" % n, p, rr, rb, None, steps, dict(seed=seed))


@dataclass
class Job:
    """One design-sweep request of the serving workload."""
    job_id: int
    arrival: float      # seconds since stream start
    side: int
    phi_v: float
    tau: float
    A: float
    nc_strength: float
    steps: int
    seed: int

    def params(self, storage=F16) -> dict:
        n = self.side
        return base_params(n, n, n, storage=storage, tau_r=self.tau, tau_b=self.tau, A=self.A,
                           beta=0.7, nc_strength=self.nc_strength, nc_range=2, nc_hmin=2.0)

    def droplets(self):
        """Droplet list of the job's emulsion (RSA with a bounded number of
        draws per droplet, radii U[6, min(12, side/4)])."""
        rng = np.random.default_rng(self.seed)
        n = self.side
        return emulsion(rng, (n, n, n), self.phi_v, 6.0, min(12.0, n / 4.0), attempts=1024)

    @property
    def sites(self) -> int:
        return self.side ** 3

    def workload(self, storage=F16) -> Workload:
        n = self.side
        cen, rad, info = self.droplets()
        phi0 = droplet_phase((n, n, n), cen, rad)
        rr, rb = split_components(phi0, 1.0)
        p = base_params(n, n, n, storage=storage, tau_r=self.tau, tau_b=self.tau, A=self.A,
                        beta=0.7, nc_strength=self.nc_strength, nc_range=2, nc_hmin=2.0)
        return Workload("job%d_%d^3" % (self.job_id, n), p, rr, rb, None, self.steps, info)


def job_stream(seed=0, n_jobs=2000, rate=40.0, sides=(32, 48, 64, 96, 128), steps=500):
    """Poisson arrivals at ``rate`` jobs/s; per-job parameters uniform in the
    ranges of the design sweep."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_jobs))
    jobs = []
    for k in range(n_jobs):
        jobs.append(Job(job_id=k, arrival=float(t[k]), side=int(rng.choice(sides)),
                        phi_v=float(rng.uniform(0.1, 0.5)), tau=float(rng.uniform(0.6, 1.2)),
                        A=float(rng.uniform(0.002, 0.02)),
                        nc_strength=float(rng.uniform(0.0, 0.05)), steps=steps,
                        seed=int(rng.integers(0, 2**31 - 1))))
    return jobs


# ---------------------------------------------------------------------------
# Small physics set-ups used by the tests
# ---------------------------------------------------------------------------

def channel(H=16, nx=1, nz=1, force=1e-5, tau=1.0, storage=F64) -> Workload:
    """Single-phase plane channel (walls at y = -1/2 and H - 1/2)."""
    shape = (nz, H, nx)
    rr = np.ones(shape)
    rb = np.zeros(shape)
    p = base_params(nx, H, nz, bc=(0, 1, 0), storage=storage, tau_r=tau, tau_b=tau,
                    body_force=(force, 0.0, 0.0))
    return Workload("channel_H%d" % H, p, rr, rb)


def shear_wave(L=32, U=1e-3, tau_r=1.0, tau_b=1.0, red_fraction=1.0, storage=F64) -> Workload:
    """u_x = U sin(2 pi y / L) on a 1 x L x 1 periodic lattice with a uniform
    mixture of the given red fraction."""
    shape = (1, L, 1)
    y = np.arange(L, dtype=np.float64)
    u = np.zeros((3,) + shape)
    u[0, 0, :, 0] = U * np.sin(2 * math.pi * y / L)
    rr = np.full(shape, red_fraction)
    rb = np.full(shape, 1.0 - red_fraction)
    p = base_params(1, L, 1, storage=storage, tau_r=tau_r, tau_b=tau_b)
    return Workload("shear_wave_L%d" % L, p, rr, rb, u)


def two_droplets(n=(48, 32, 1), R=8.0, gap=2.0, A=0.01, tau=1.0, nc_strength=0.0, nc_range=2,
                 nc_hmin=2.0, storage=F64) -> Workload:
    """Two equal droplets (discs when nz = 1) on the x axis whose tanh
    profiles' zero level sets are ``gap`` sites apart, mirror symmetric about
    the box centre."""
    nx, ny, nz = n
    cx, cy, cz = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    off = R + gap / 2.0
    cen = [(cx - off, cy, cz), (cx + off, cy, cz)]
    if nz == 1:
        cen = [(c[0], c[1], 0.0) for c in cen]
    phi0 = _droplet_phase_2d(nz, ny, nx, cen, [R, R]) if nz == 1 else \
        droplet_phase((nz, ny, nx), cen, [R, R])
    rr, rb = split_components(phi0, 1.0)
    p = base_params(nx, ny, nz, storage=storage, tau_r=tau, tau_b=tau, A=A,
                    nc_strength=nc_strength, nc_range=nc_range, nc_hmin=nc_hmin)
    return Workload("two_droplets_gap%g" % gap, p, rr, rb)


def _droplet_phase_2d(nz, ny, nx, centres, radii, width=2.0):
    """Discs (cylinders along z) for quasi-2D set-ups."""
    y = np.arange(ny, dtype=np.float64)[:, None]
    x = np.arange(nx, dtype=np.float64)[None, :]
    phi = np.full((ny, nx), -1.0)
    for c, R in zip(centres, radii):
        dx = _axis_dist(x, c[0], nx, True)
        dy = _axis_dist(y, c[1], ny, True)
        phi = np.maximum(phi, np.tanh((R - np.sqrt(dx ** 2 + dy ** 2)) / width))
    return np.broadcast_to(phi, (nz, ny, nx)).copy()


def disc(n=48, R=10.0, A=0.01, tau=1.0, storage=F64) -> Workload:
    """A single disc (a cylinder along z) in an n x n x 1 periodic box."""
    c = (n - 1) / 2.0
    phi0 = _droplet_phase_2d(1, n, n, [(c, c, 0.0)], [R])
    rr, rb = split_components(phi0, 1.0)
    p = base_params(n, n, 1, storage=storage, tau_r=tau, tau_b=tau, A=A)
    return Workload("disc_R%g" % R, p, rr, rb)


def sphere(n=48, R=10.0, A=0.01, tau=1.0, storage=F64) -> Workload:
    c = (n - 1) / 2.0
    phi0 = droplet_phase((n, n, n), [(c, c, c)], [R])
    rr, rb = split_components(phi0, 1.0)
    p = base_params(n, n, n, storage=storage, tau_r=tau, tau_b=tau, A=A)
    return Workload("sphere_R%g" % R, p, rr, rb)


def random_state(seed, shape, amp=0.05):
    """Arbitrary positive densities and small velocities for generic tests."""
    rng = np.random.default_rng(seed)
    phi0 = np.tanh(rng.normal(0.0, 1.0, size=shape))
    rho0 = 1.0 + amp * rng.uniform(-1, 1, size=shape)
    rr, rb = split_components(phi0, rho0)
    u = amp * 0.2 * rng.uniform(-1, 1, size=(3,) + tuple(shape))
    return rr, rb, u

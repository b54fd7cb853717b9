"""FP64 CPU oracle for the two-component colour-gradient D3Q19 update.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports
this module and this module imports nothing from the GPU library.

Thin ctypes marshalling around ``lb_oracle.c`` (which holds every piece of
arithmetic, each function citing the passage of arXiv 2005.12764 it follows).
Arrays are numpy float64, C-contiguous.  Populations are shaped
``(2, 19, nz, ny, nx)`` (component red/blue, direction, z, y, x); vector fields
are ``(3, nz, ny, nx)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

Q = 19


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_tables.argtypes = [ip, dp, ip, dp]
        L.orc_feq.argtypes = [ctypes.c_double, dp, dp]
        L.orc_omega.argtypes = [ctypes.c_double] * 4
        L.orc_omega.restype = ctypes.c_double
        L.orc_bgk_edm.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        L.orc_perturbation.argtypes = [ctypes.c_double, dp, ctypes.c_double, dp]
        L.orc_recolour.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp,
                                   ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_collide_site.argtypes = [dp, dp, dp, dp, dp, dp, dp]
        L.orc_init.argtypes = [dp, dp, dp, dp, dp]
        L.orc_moments.argtypes = [dp, dp, dp, dp, dp]
        L.orc_phase_gradient.argtypes = [dp, dp, dp]
        L.orc_nc_amplitude.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.orc_nc_amplitude.restype = ctypes.c_double
        L.orc_nearcontact.argtypes = [dp, dp, dp]
        L.orc_collide.argtypes = [dp, dp, dp, dp, dp, dp]
        L.orc_sc_force.argtypes = [dp, dp, dp, dp, dp]
        L.orc_sc_collide_site.argtypes = [dp, dp, dp, dp, dp, dp, dp]
        L.orc_stream.argtypes = [dp, dp, dp]
        L.orc_step.argtypes = [dp, dp, dp, ctypes.c_int]
        L.orc_phase_field.argtypes = [dp, dp, dp]
        L.orc_korteweg.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_block_average.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Params:
    """Parameters of one lattice; mirrors the quantities the paper names."""
    nx: int
    ny: int
    nz: int
    bc: tuple = (0, 0, 0)          # 0 periodic, 1 halfway bounce-back walls
    tau_r: float = 1.0
    tau_b: float = 1.0
    A: float = 0.0                 # surface-tension perturbation amplitude
    beta: float = 0.7              # recolouring segregation
    nc_strength: float = 0.0       # near-contact strength A
    nc_range: int = 0              # probe range K
    nc_hmin: float = 2.0           # h_min
    body_force: tuple = (0.0, 0.0, 0.0)
    eps_g: float = 1e-12
    g_iface: float = 0.05
    wall_velocity: tuple = ((0.0, 0.0, 0.0),) * 6   # faces -x, +x, -y, +y, -z, +z
    model: int = 0                 # interface model: 0 colour gradient, 1 Shan-Chen
    g_sc: float = 0.0              # Shan-Chen coupling G_C (> 0 repulsive)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def vec(self) -> np.ndarray:
        return np.array([self.nx, self.ny, self.nz, *self.bc, self.tau_r, self.tau_b,
                         self.A, self.beta, self.nc_strength, self.nc_range, self.nc_hmin,
                         *self.body_force, self.eps_g, self.g_iface,
                         *np.asarray(self.wall_velocity, dtype=np.float64).reshape(18),
                         self.model, self.g_sc],
                        dtype=np.float64)


def params_from_dict(p: dict, eps_g=None, g_iface: float = 0.05) -> Params:
    """Oracle parameters for a parameter dict with the library's keys (the
    same physical quantities); eps_g defaults to 1e-12 for FP64 storage
    (storage 0) and 1e-6 otherwise, the thresholds the GPU library uses."""
    if eps_g is None:
        eps_g = 1e-12 if int(p.get("storage", 0)) == 0 else 1e-6
    return Params(nx=p["nx"], ny=p["ny"], nz=p["nz"], bc=tuple(p["bc"]),
                  tau_r=p["tau_r"], tau_b=p["tau_b"], A=p["A"], beta=p["beta"],
                  nc_strength=p["nc_strength"], nc_range=p["nc_range"],
                  nc_hmin=p["nc_hmin"], body_force=tuple(p["body_force"]),
                  eps_g=eps_g, g_iface=g_iface,
                  wall_velocity=tuple(map(tuple, p.get("wall_velocity", ((0.0, 0.0, 0.0),) * 6))),
                  model=int(p.get("model", 0)), g_sc=float(p.get("g_sc", 0.0)))


def tables():
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    bp = np.zeros(Q)
    ip = ctypes.POINTER(ctypes.c_int)
    lib().orc_tables(c.ctypes.data_as(ip), _p(w), opp.ctypes.data_as(ip), _p(bp))
    return c, w, opp, bp


def feq(rho, u):
    out = np.zeros(Q)
    lib().orc_feq(float(rho), _p(_f64(u)), _p(out))
    return out


def omega(tau_r, tau_b, rho_r, rho_b):
    return lib().orc_omega(tau_r, tau_b, rho_r, rho_b)


def bgk_edm(om, rho_k, u, du, fk):
    out = np.zeros(Q)
    lib().orc_bgk_edm(float(om), float(rho_k), _p(_f64(u)), _p(_f64(du)), _p(_f64(fk)), _p(out))
    return out


def perturbation(A, G, eps_g=1e-12):
    out = np.zeros(Q)
    lib().orc_perturbation(float(A), _p(_f64(G)), float(eps_g), _p(out))
    return out


def recolour(rho_r, rho_b, fstar, G, beta, eps_g=1e-12):
    outr, outb = np.zeros(Q), np.zeros(Q)
    lib().orc_recolour(float(rho_r), float(rho_b), _p(_f64(fstar)), _p(_f64(G)),
                       float(beta), float(eps_g), _p(outr), _p(outb))
    return outr, outb


def collide_site(prm: Params, fr, fb, G, F):
    outr, outb = np.zeros(Q), np.zeros(Q)
    lib().orc_collide_site(_p(prm.vec()), _p(_f64(fr)), _p(_f64(fb)), _p(_f64(G)),
                           _p(_f64(F)), _p(outr), _p(outb))
    return outr, outb


def nc_amplitude(strength, hmin, K, h):
    return lib().orc_nc_amplitude(float(strength), float(hmin), int(K), int(h))


def init(prm: Params, rho_r, rho_b, u=None):
    f = np.zeros((2, Q) + prm.shape)
    lib().orc_init(_p(prm.vec()), _p(_f64(rho_r)), _p(_f64(rho_b)),
                   _p(_f64(u)) if u is not None else None, _p(f))
    return f


def moments(prm: Params, f):
    rr = np.zeros(prm.shape)
    rb = np.zeros(prm.shape)
    j = np.zeros((3,) + prm.shape)
    lib().orc_moments(_p(prm.vec()), _p(_f64(f)), _p(rr), _p(rb), _p(j))
    return rr, rb, j


def phase_gradient(prm: Params, phi):
    G = np.zeros((3,) + prm.shape)
    lib().orc_phase_gradient(_p(prm.vec()), _p(_f64(phi)), _p(G))
    return G


def phase_field(prm: Params, f):
    phi = np.zeros(prm.shape)
    lib().orc_phase_field(_p(prm.vec()), _p(_f64(f)), _p(phi))
    return phi


def korteweg(prm: Params, phi, lam: float):
    """Korteweg tensor of the field phi, (6, nz, ny, nx): xx, yy, zz, xy, xz, yz."""
    K = np.zeros((6,) + prm.shape)
    lib().orc_korteweg(_p(prm.vec()), _p(_f64(phi)), float(lam), _p(K))
    return K


def block_average(prm: Params, field, b: int):
    """Means over b x b x b blocks of (ncomp, nz, ny, nx) or (nz, ny, nx) fields."""
    a = _f64(field)
    one = a.ndim == 3
    a = a.reshape((1,) + prm.shape) if one else a
    nz, ny, nx = prm.shape
    if nx % b or ny % b or nz % b:
        raise ValueError("lattice extents must be multiples of the block size")
    out = np.zeros((a.shape[0], nz // b, ny // b, nx // b))
    lib().orc_block_average(_p(prm.vec()), _p(np.ascontiguousarray(a)), a.shape[0], int(b), _p(out))
    return out[0] if one else out


def nearcontact(prm: Params, G):
    F = np.zeros((3,) + prm.shape)
    lib().orc_nearcontact(_p(prm.vec()), _p(_f64(G)), _p(F))
    return F


def sc_force(prm: Params, rho_r, rho_b):
    """Shan-Chen force densities (F^r, F^b), each (3, nz, ny, nx)."""
    Fr = np.zeros((3,) + prm.shape)
    Fb = np.zeros((3,) + prm.shape)
    lib().orc_sc_force(_p(prm.vec()), _p(_f64(rho_r)), _p(_f64(rho_b)), _p(Fr), _p(Fb))
    return Fr, Fb


def sc_collide_site(prm: Params, fr, fb, Fr, Fb):
    outr, outb = np.zeros(Q), np.zeros(Q)
    lib().orc_sc_collide_site(_p(prm.vec()), _p(_f64(fr)), _p(_f64(fb)), _p(_f64(Fr)),
                              _p(_f64(Fb)), _p(outr), _p(outb))
    return outr, outb


def collide(prm: Params, f, want_fields: bool = False):
    """Collision of the whole lattice.  With want_fields, also the phase
    field, the colour gradient G and the near-contact force (Shan-Chen model:
    F^r and F^b in place of G and the near-contact force)."""
    post = np.zeros_like(_f64(f))
    if want_fields:
        phi = np.zeros(prm.shape)
        G = np.zeros((3,) + prm.shape)
        Fn = np.zeros((3,) + prm.shape)
        lib().orc_collide(_p(prm.vec()), _p(_f64(f)), _p(post), _p(phi), _p(G), _p(Fn))
        return post, phi, G, Fn
    lib().orc_collide(_p(prm.vec()), _p(_f64(f)), _p(post), None, None, None)
    return post


def stream(prm: Params, fpost):
    out = np.empty_like(_f64(fpost))
    lib().orc_stream(_p(prm.vec()), _p(_f64(fpost)), _p(out))
    return out


def step(prm: Params, f, n: int = 1):
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_step(_p(prm.vec()), _p(f), _p(out), int(n))
    return out


def threads() -> int:
    return lib().orc_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))

"""ctypes binding of liblb.so (include/lb.h), argument marshalling only.

Every step of the update runs in the library's HIP kernels; this module only
converts Python/numpy/torch arguments to the C ABI.  Importing it does not load
the library; the first call does, and raises if the library is not built.
Host arrays are numpy; device arrays are torch CUDA (HIP) tensors, passed by
``data_ptr()``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .workloads import F64, F32, F16, BF16  # storage codes  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblb.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ESTATE = 0, -1, -2, -3, -4
KERNEL_AUTO, KERNEL_TWOPASS, KERNEL_FUSED = 0, 1, 2
MODEL_COLOUR_GRADIENT, MODEL_SHAN_CHEN = 0, 1
DTYPE_F64, DTYPE_F32 = 0, 1
MAX_NC_RANGE = 4
Q = 19


class LbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("liblb error %d: %s" % (code, msg))
        self.code = code


class lb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 3),
        ("storage", ctypes.c_int32), ("kernel", ctypes.c_int32),
        ("tau_r", ctypes.c_double), ("tau_b", ctypes.c_double),
        ("A", ctypes.c_double), ("beta", ctypes.c_double),
        ("nc_strength", ctypes.c_double),
        ("nc_range", ctypes.c_int32), ("scale_log2", ctypes.c_int32),
        ("nc_hmin", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("eps_g", ctypes.c_double), ("g_iface", ctypes.c_double),
        ("wall_velocity", (ctypes.c_double * 3) * 6),
        ("model", ctypes.c_int32), ("g_sc", ctypes.c_double),
    ]


def make_params(p: dict) -> lb_params:
    """lb_params from a parameter dict (keys as in workloads.base_params)."""
    s = lb_params()
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    for a in range(3):
        s.bc[a] = int(p.get("bc", (0, 0, 0))[a])
        s.body_force[a] = float(p.get("body_force", (0.0, 0.0, 0.0))[a])
    s.storage = int(p.get("storage", F32))
    s.kernel = int(p.get("kernel", KERNEL_AUTO))
    s.tau_r, s.tau_b = float(p["tau_r"]), float(p["tau_b"])
    s.A, s.beta = float(p.get("A", 0.0)), float(p.get("beta", 0.7))
    s.nc_strength = float(p.get("nc_strength", 0.0))
    s.nc_range = int(p.get("nc_range", 0))
    s.scale_log2 = int(p.get("scale_log2", 0))
    s.nc_hmin = float(p.get("nc_hmin", 2.0))
    s.eps_g = float(p.get("eps_g", 0.0))
    s.g_iface = float(p.get("g_iface", 0.0))
    s.model = int(p.get("model", MODEL_COLOUR_GRADIENT))
    s.g_sc = float(p.get("g_sc", 0.0))
    uw = p.get("wall_velocity")
    if uw is not None:
        uw = np.asarray(uw, dtype=np.float64).reshape(6, 3)
        for f in range(6):
            for a in range(3):
                s.wall_velocity[f][a] = float(uw[f, a])
    return s


_lib = None


def lib():
    """Load liblb.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblb.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch ships its own HIP runtime under the same soname; loading torch first
    # makes liblb.so bind to that one, so the process holds a single runtime and
    # torch streams and device pointers are valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(lb_params)
    sig = {
        "lb_create": ([pp, vp, ctypes.POINTER(vp)], i32),
        "lb_init_fields": ([vp, vp, vp, vp, i32, i32], i32),
        "lb_step": ([vp, i32], i32),
        "lb_moments": ([vp, vp, vp, vp, i32, i32, dp], i32),
        "lb_korteweg": ([vp, ctypes.c_double, i32, vp, vp, i32, i32, i32], i32),
        "lb_set_tiles": ([i32, i32, i32, i32], i32),
        "lb_step_timed": ([vp, i32, dp], i32),
        "lb_get_state": ([vp, vp, i32, i32], i32),
        "lb_set_state": ([vp, vp, i32, i32], i32),
        "lb_state_bytes": ([vp], i64),
        "lb_save_raw": ([vp, vp, i32], i32),
        "lb_load_raw": ([vp, vp, i32], i32),
        "lb_step_count": ([vp], i64),
        "lb_kernel_in_use": ([vp], i32),
        "lb_destroy": ([vp], i32),
        "lb_last_error": ([], ctypes.c_char_p),
        "lb_footprint_bytes": ([pp], i64),
        "lb_pattern_ms": ([pp, i32, dp], i32),
        "lb_batch_create": ([i32, i64, i32, i32, vp, ctypes.POINTER(vp)], i32),
        "lb_batch_add": ([vp, pp, vp, vp, vp, i32, i32, i64, ctypes.POINTER(i32)], i32),
        "lb_batch_add_droplets": ([vp, pp, dp, dp, i32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, i64, ctypes.POINTER(i32)], i32),
        "lb_batch_job_bytes": ([pp], i64),
        "lb_init_droplets": ([vp, dp, dp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double], i32),
        "lb_batch_remove": ([vp, i32], i32),
        "lb_batch_step": ([vp, i32], i32),
        "lb_batch_moments": ([vp, i32, vp, vp, vp, i32, i32, dp], i32),
        "lb_batch_get_state": ([vp, i32, vp, i32, i32], i32),
        "lb_batch_job_steps": ([vp, i32], i64),
        "lb_batch_free_bytes": ([vp], i64),
        "lb_batch_destroy": ([vp], i32),
        "lb_state_totals_noalloc": ([pp, vp, i32, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc < 0:
        raise LbError(rc, lib().lb_last_error().decode())
    return rc


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _arg(a, dtype_code: Optional[int] = None):
    """(pointer, on_device, dtype_code, keepalive) of a numpy array or torch tensor."""
    if a is None:
        return None, 0, dtype_code, None
    if _is_torch(a):
        import torch
        if not a.is_contiguous():
            raise ValueError("device tensors must be contiguous")
        code = {torch.float64: DTYPE_F64, torch.float32: DTYPE_F32}[a.dtype]
        return ctypes.c_void_p(a.data_ptr()), int(a.is_cuda), code, a
    arr = np.ascontiguousarray(a)
    if arr.dtype not in (np.float64, np.float32):
        arr = arr.astype(np.float64)
    code = DTYPE_F64 if arr.dtype == np.float64 else DTYPE_F32
    return ctypes.c_void_p(arr.ctypes.data), 0, code, arr


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        return ctypes.c_void_p(None)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ----------------------------------------------------------------------------
# C-ABI names
# ----------------------------------------------------------------------------

def lb_create(params: dict, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    prm = make_params(params)
    _check(lib().lb_create(ctypes.byref(prm), _stream_ptr(stream), ctypes.byref(h)))
    return h


def lb_init_fields(h, rho_r, rho_b, u=None) -> None:
    pr, dev, code, k1 = _arg(rho_r)
    pb, dev2, code2, k2 = _arg(rho_b, code)
    pu, dev3, code3, k3 = _arg(u, code)
    if code2 != code or (u is not None and code3 != code) or dev2 != dev or (u is not None and dev3 != dev):
        raise ValueError("rho_r, rho_b and u must share dtype and device")
    _check(lib().lb_init_fields(h, pr, pb, pu, code, dev))


def _droplets(centres, radii):
    c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 3))
    r = np.ascontiguousarray(np.asarray(radii, dtype=np.float64).reshape(-1))
    if len(c) != len(r):
        raise ValueError("centres and radii differ in length")
    dp = ctypes.POINTER(ctypes.c_double)
    return c, r, c.ctypes.data_as(dp), r.ctypes.data_as(dp)


def lb_init_droplets(h, centres, radii, width=2.0, background=-1.0, rho0=1.0) -> None:
    c, r, pc, pr = _droplets(centres, radii)
    _check(lib().lb_init_droplets(h, pc, pr, len(r), float(width), float(background), float(rho0)))


def lb_step(h, n: int = 1) -> None:
    _check(lib().lb_step(h, int(n)))


def lb_step_timed(h, n: int):
    """Run n steps timing each pass with HIP events; returns mean ms per step
    of (phase pass, collide/fused pass, whole step)."""
    out = (ctypes.c_double * 3)()
    _check(lib().lb_step_timed(h, int(n), ctypes.cast(out, ctypes.POINTER(ctypes.c_double))))
    return tuple(out[:])


def lb_moments(h, rho_r=None, rho_b=None, mom=None, want_totals: bool = False):
    """Fill the given output arrays (numpy host or torch device, same dtype);
    return the 7 compensated totals (sum + correction) if requested."""
    outs = [o for o in (rho_r, rho_b, mom) if o is not None]
    code, dev = DTYPE_F64, 0
    ptrs = []
    for o in (rho_r, rho_b, mom):
        if o is None:
            ptrs.append(None)
            continue
        if _is_torch(o):
            p, dev, code, _ = _arg(o)
        else:
            if not (isinstance(o, np.ndarray) and o.flags.c_contiguous):
                raise ValueError("host outputs must be C-contiguous numpy arrays")
            code = DTYPE_F64 if o.dtype == np.float64 else DTYPE_F32
            p = ctypes.c_void_p(o.ctypes.data)
        ptrs.append(p)
    tot = (ctypes.c_double * 14)() if want_totals else None
    _check(lib().lb_moments(h, ptrs[0], ptrs[1], ptrs[2], code, dev,
                            ctypes.cast(tot, ctypes.POINTER(ctypes.c_double)) if tot else None))
    if want_totals:
        t = np.array(tot[:], dtype=np.float64).reshape(7, 2)
        return t
    return None


def lb_state_totals_noalloc(params: dict, f, totals, stream=None) -> None:
    """The 7 compensated totals (sum, correction pairs) of a population
    state f ([2][19][nz][ny][nx] torch device tensor, float64 or float32, the
    layout of lb_get_state) into `totals` (torch float64 device tensor of 14),
    ordered on `stream`; the library allocates nothing for it."""
    if not (_is_torch(f) and f.is_cuda and _is_torch(totals) and totals.is_cuda):
        raise ValueError("f and totals must be device tensors")
    if totals.dtype != torch_float64() or totals.numel() != 14 or not totals.is_contiguous():
        raise ValueError("totals must be a contiguous float64 tensor of 14 values")
    pf, _, code, _ = _arg(f)
    prm = make_params(params)
    _check(lib().lb_state_totals_noalloc(ctypes.byref(prm), pf, code, ctypes.c_void_p(totals.data_ptr()),
                                         _stream_ptr(stream)))


def torch_float64():
    import torch
    return torch.float64


TILES_PHASE, TILES_COLLIDE, TILES_ONE_READ, TILES_BATCH = 0, 1, 2, 3


def lb_set_tiles(kind: int, storage: int, ty: int = 0, tz: int = 0) -> None:
    """Tile rows / chunk planes of one tile kind for one storage (0 = default)."""
    _check(lib().lb_set_tiles(int(kind), int(storage), int(ty), int(tz)))


def lb_korteweg(h, lam: float, b: int, k_blocks=None, phi_blocks=None, accumulate: bool = False) -> None:
    """Block averages of the Korteweg tensor (6, nz/b, ny/b, nx/b) and of phi
    (nz/b, ny/b, nx/b) into the given outputs (numpy host or torch device,
    same dtype; either may be None)."""
    code, dev, ptrs = DTYPE_F64, 0, []
    for o in (k_blocks, phi_blocks):
        if o is None:
            ptrs.append(None)
            continue
        if _is_torch(o):
            p, dev, code, _ = _arg(o)
        else:
            if not (isinstance(o, np.ndarray) and o.flags.c_contiguous):
                raise ValueError("host outputs must be C-contiguous numpy arrays")
            code = DTYPE_F64 if o.dtype == np.float64 else DTYPE_F32
            p = ctypes.c_void_p(o.ctypes.data)
        ptrs.append(p)
    _check(lib().lb_korteweg(h, float(lam), int(b), ptrs[0], ptrs[1], code, dev, int(bool(accumulate))))


def lb_get_state(h, out) -> None:
    p, dev, code, _ = _arg(out) if _is_torch(out) else (ctypes.c_void_p(out.ctypes.data), 0,
                                                         DTYPE_F64 if out.dtype == np.float64 else DTYPE_F32, out)
    _check(lib().lb_get_state(h, p, code, dev))


def lb_set_state(h, f) -> None:
    p, dev, code, keep = _arg(f)
    _check(lib().lb_set_state(h, p, code, dev))


def lb_destroy(h) -> None:
    _check(lib().lb_destroy(h))


def lb_last_error() -> str:
    return lib().lb_last_error().decode()


def lb_footprint_bytes(params: dict) -> int:
    prm = make_params(params)
    return int(lib().lb_footprint_bytes(ctypes.byref(prm)))


def lb_pattern_ms(params: dict, reps: int = 20) -> float:
    """Average duration (ms) of a launch of the FP32 one-read step's memory
    access pattern without arithmetic on a periodic lattice of these sizes
    (lb_pattern_ms)."""
    prm = make_params(params)
    out = ctypes.c_double(0.0)
    _check(lib().lb_pattern_ms(ctypes.byref(prm), int(reps), ctypes.byref(out)))
    return float(out.value)


# ----------------------------------------------------------------------------
# Batched form
# ----------------------------------------------------------------------------

def lb_batch_job_bytes(params: dict) -> int:
    prm = make_params(params)
    return int(lib().lb_batch_job_bytes(ctypes.byref(prm)))


class Batch:
    """Many independent lattices advanced together by the batched step."""

    def __init__(self, max_jobs: int, arena_bytes: int, storage: int = F16, graph_steps: int = 50,
                 stream=None):
        self.storage = int(storage)
        self.h = ctypes.c_void_p()
        _check(lib().lb_batch_create(int(max_jobs), int(arena_bytes), self.storage, int(graph_steps),
                                     _stream_ptr(stream), ctypes.byref(self.h)))
        self.shapes = {}

    def add(self, params: dict, rho_r, rho_b, u=None, steps: int = 0) -> int:
        prm = make_params(dict(params, storage=self.storage))
        pr, dev, code, k1 = _arg(rho_r)
        pb, _, _, k2 = _arg(rho_b, code)
        pu, _, _, k3 = _arg(u, code)
        slot = ctypes.c_int32()
        _check(lib().lb_batch_add(self.h, ctypes.byref(prm), pr, pb, pu, code, dev, int(steps),
                                  ctypes.byref(slot)))
        self.shapes[slot.value] = (prm.nz, prm.ny, prm.nx)
        return slot.value

    def add_droplets(self, params: dict, centres, radii, steps: int, width=2.0, background=-1.0,
                     rho0=1.0) -> int:
        prm = make_params(dict(params, storage=self.storage))
        c, r, pc, pr = _droplets(centres, radii)
        slot = ctypes.c_int32()
        _check(lib().lb_batch_add_droplets(self.h, ctypes.byref(prm), pc, pr, len(r), float(width),
                                           float(background), float(rho0), int(steps),
                                           ctypes.byref(slot)))
        self.shapes[slot.value] = (prm.nz, prm.ny, prm.nx)
        return slot.value

    def remove(self, slot: int) -> None:
        _check(lib().lb_batch_remove(self.h, int(slot)))
        self.shapes.pop(slot, None)

    def step(self, n: int) -> None:
        _check(lib().lb_batch_step(self.h, int(n)))

    def job_steps(self, slot: int) -> int:
        return int(lib().lb_batch_job_steps(self.h, int(slot)))

    def free_bytes(self) -> int:
        return int(lib().lb_batch_free_bytes(self.h))

    def totals(self, slot: int) -> np.ndarray:
        tot = (ctypes.c_double * 14)()
        _check(lib().lb_batch_moments(self.h, int(slot), None, None, None, DTYPE_F64, 0,
                                      ctypes.cast(tot, ctypes.POINTER(ctypes.c_double))))
        return np.array(tot[:], dtype=np.float64).reshape(7, 2)

    def moments(self, slot: int):
        shape = self.shapes[slot]
        rr, rb, j = np.empty(shape), np.empty(shape), np.empty((3,) + shape)
        vp = ctypes.c_void_p
        _check(lib().lb_batch_moments(self.h, int(slot), vp(rr.ctypes.data), vp(rb.ctypes.data),
                                      vp(j.ctypes.data), DTYPE_F64, 0, None))
        return rr, rb, j

    def state(self, slot: int, dtype=np.float64) -> np.ndarray:
        out = np.empty((2, Q) + self.shapes[slot], dtype=dtype)
        code = DTYPE_F64 if out.dtype == np.float64 else DTYPE_F32
        _check(lib().lb_batch_get_state(self.h, int(slot), ctypes.c_void_p(out.ctypes.data), code, 0))
        return out

    def close(self):
        if self.h is not None and self.h.value:
            _check(lib().lb_batch_destroy(self.h))
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# Convenience wrapper
# ----------------------------------------------------------------------------

class Lattice:
    """One lattice owned by the library.  Host-side results are numpy arrays
    shaped (nz, ny, nx) / (3, nz, ny, nx) / (2, 19, nz, ny, nx)."""

    def __init__(self, params: dict, stream=None):
        self.params = dict(params)
        self.shape = (int(params["nz"]), int(params["ny"]), int(params["nx"]))
        self.N = int(np.prod(self.shape))
        self.h = lb_create(self.params, stream)

    def init(self, rho_r, rho_b, u=None):
        lb_init_fields(self.h, rho_r, rho_b, u)
        return self

    def init_droplets(self, centres, radii, width=2.0, background=-1.0, rho0=1.0):
        lb_init_droplets(self.h, centres, radii, width, background, rho0)
        return self

    def step(self, n: int = 1):
        lb_step(self.h, n)
        return self

    def moments(self):
        rr = np.empty(self.shape)
        rb = np.empty(self.shape)
        j = np.empty((3,) + self.shape)
        lb_moments(self.h, rr, rb, j)
        return rr, rb, j

    def totals(self):
        return lb_moments(self.h, want_totals=True)

    def korteweg(self, lam: float, b: int):
        """Host FP64 block averages of the Korteweg tensor and of phi."""
        nz, ny, nx = self.shape
        K = np.empty((6, nz // b, ny // b, nx // b))
        phi = np.empty((nz // b, ny // b, nx // b))
        lb_korteweg(self.h, lam, b, K, phi)
        return K, phi

    def state(self, dtype=np.float64):
        out = np.empty((2, Q) + self.shape, dtype=dtype)
        lb_get_state(self.h, out)
        return out

    def set_state(self, f):
        lb_set_state(self.h, f)

    @property
    def steps(self) -> int:
        return int(lib().lb_step_count(self.h))

    @property
    def kernel(self) -> int:
        return int(lib().lb_kernel_in_use(self.h))

    def state_bytes(self) -> int:
        return int(lib().lb_state_bytes(self.h))

    def save_raw(self) -> np.ndarray:
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        _check(lib().lb_save_raw(self.h, ctypes.c_void_p(buf.ctypes.data), 0))
        return buf

    def load_raw(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(lib().lb_load_raw(self.h, ctypes.c_void_p(buf.ctypes.data), 0))

    def close(self):
        if self.h is not None:
            lb_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Tile-shape autotuner for the library's tile kernels.

For one storage type and one box class (lattice size), it times every
candidate tile shape (rows of a 64-wide tile, planes of the z chunk a
workgroup marches) of each tile kind on a seeded synthetic emulsion of that
size, keeps the fastest, and records it in a JSON cache keyed by
(architecture, storage, kind, box class).  ``apply`` hands the cached shapes
to the library (``lb_set_tiles``).  The library's built-in defaults are the
shapes this tuner picked for the 256^3 emulsion on MI355X.

Kinds: the one-read step (timed as a whole step), the two passes of the
two-pass step (each pass timed on its own), and the batched step (timed per
step over a mix of jobs).  The timings use HIP events around the kernels
(``lb_step_timed``) or around a batch's graph replays.

    python -m paper_2005_12764_amd.autotune --n 128 --storage f32,f16 --batch f16 --out tiles.json
"""
from __future__ import annotations

import argparse
import json
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Tuple

from . import lb
from . import workloads as W

KIND_NAME = {lb.TILES_PHASE: "phase", lb.TILES_COLLIDE: "collide", lb.TILES_ONE_READ: "one_read",
             lb.TILES_BATCH: "batch"}
STORAGE_NAME = {W.F64: "f64", W.F32: "f32", W.F16: "f16", W.BF16: "bf16"}

# candidate (rows, planes); planes 0 = the library's choice for the lattice
CANDIDATES: Dict[int, List[Tuple[int, int]]] = {
    lb.TILES_ONE_READ: [(ty, tz) for ty in (4, 8, 16) for tz in (0, 16, 32, 64)],
    lb.TILES_COLLIDE: [(ty, tz) for ty in (2, 4, 8) for tz in (0, 16, 32, 64)],
    lb.TILES_PHASE: [(ty, tz) for ty in (4, 8, 16) for tz in (0, 16, 32, 64)],
    lb.TILES_BATCH: [(ty, tz) for ty in (4, 8) for tz in (16, 32, 64)],
}


def box_class(sites: int) -> str:
    """Size class of a lattice (or of a batch's mean job)."""
    if sites <= 1 << 18:
        return "small"
    if sites <= 1 << 22:
        return "medium"
    return "large"


def cache_key(arch: str, storage: int, kind: int, cls: str) -> str:
    return "%s/%s/%s/%s" % (arch, STORAGE_NAME[storage], KIND_NAME[kind], cls)


def pick(timer: Callable[[int, int], float], candidates: Iterable[Tuple[int, int]]):
    """Time every candidate with timer(ty, tz) -> ms (None = not runnable);
    return the fastest (ty, tz, ms) and every timing, in candidate order."""
    results = []
    best = None
    for ty, tz in candidates:
        ms = timer(ty, tz)
        results.append({"ty": ty, "tz": tz, "ms": ms})
        if ms is not None and (best is None or ms < best[2]):
            best = (ty, tz, ms)
    if best is None:
        raise RuntimeError("no candidate tile shape ran")
    return best, results


def load(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(cache: dict, path: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(cache: dict, arch: str, storage: int, sites: int, kinds=None) -> Dict[int, Tuple[int, int]]:
    """Set the cached tile shapes of a storage and box class in the library;
    returns what was set, by kind."""
    done = {}
    for kind in (kinds or KIND_NAME):
        e = cache.get(cache_key(arch, storage, kind, box_class(sites)))
        if e:
            lb.lb_set_tiles(kind, storage, e["ty"], e["tz"])
            done[kind] = (e["ty"], e["tz"])
    return done


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


# ------------------------------------------------------------------ timers

def _lattice_timer(w, storage: int, kind: int, steps: int, stream=None):
    """timer(ty, tz) for one tile kind of a single lattice of workload w."""
    kernel = lb.KERNEL_FUSED if kind == lb.TILES_ONE_READ else lb.KERNEL_TWOPASS
    which = {lb.TILES_ONE_READ: 2, lb.TILES_COLLIDE: 1, lb.TILES_PHASE: 0}[kind]

    def timer(ty: int, tz: int) -> Optional[float]:
        lb.lb_set_tiles(kind, storage, ty, tz)
        try:
            with lb.Lattice(dict(w.params, storage=storage, kernel=kernel), stream=stream) as L:
                L.init(w.rho_r, w.rho_b)
                L.step(2)
                return float(lb.lb_step_timed(L.h, steps)[which])
        except lb.LbError:
            return None
        finally:
            lb.lb_set_tiles(kind, storage, 0, 0)
    return timer


def _batch_timer(storage: int, jobs: list, steps: int):
    """timer(ty, tz) for the batched step over the given (params, rr, rb) jobs."""
    import torch
    total = sum(p["nx"] * p["ny"] * p["nz"] for p, _, _ in jobs)

    def timer(ty: int, tz: int) -> Optional[float]:
        lb.lb_set_tiles(lb.TILES_BATCH, storage, ty, tz)
        try:
            need = sum(lb.lb_footprint_bytes(dict(p, storage=storage, kernel=lb.KERNEL_TWOPASS))
                       for p, _, _ in jobs)
            with lb.Batch(len(jobs), int(need * 1.5) + (64 << 20), storage, graph_steps=steps) as B:
                for p, rr, rb in jobs:
                    B.add(dict(p, storage=storage), rr, rb, steps=1 << 30)
                B.step(steps)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                B.step(2 * steps)
                torch.cuda.synchronize()
                return (time.perf_counter() - t0) * 1e3 / (2 * steps)
        except lb.LbError:
            return None
        finally:
            lb.lb_set_tiles(lb.TILES_BATCH, storage, 0, 0)
    timer.sites = total
    return timer


def tune_lattice(n: int, storage: int, arch: str, cache: dict, steps: int = 20, log=print) -> dict:
    """Tune the tile kinds a lattice of side n with this storage steps with."""
    w = W.periodic_emulsion(seed=0, n=n, storage=storage)
    kinds = [lb.TILES_ONE_READ] if storage in (W.F64, W.F32) else []
    kinds += [lb.TILES_PHASE, lb.TILES_COLLIDE] if storage in (W.F16, W.BF16) else [lb.TILES_COLLIDE]
    out = {}
    for kind in kinds:
        best, res = pick(_lattice_timer(w, storage, kind, steps), CANDIDATES[kind])
        k = cache_key(arch, storage, kind, box_class(w.sites))
        cache[k] = {"ty": best[0], "tz": best[1], "ms": round(best[2], 4), "sites": w.sites,
                    "timings": res}
        out[k] = cache[k]
        log("%s: ty %d tz %d %.4f ms" % (k, best[0], best[1], best[2]))
    return out


def tune_batch(storage: int, arch: str, cache: dict, sides=(32, 48, 64, 96), copies: int = 4,
               steps: int = 10, log=print) -> dict:
    """Tune the batched step on a mix of emulsion jobs of the given sides."""
    jobs = []
    for k, s in enumerate(sides):
        w = W.periodic_emulsion(seed=k, n=s, storage=storage)
        jobs += [(w.params, w.rho_r, w.rho_b)] * copies
    timer = _batch_timer(storage, jobs, steps)
    best, res = pick(timer, CANDIDATES[lb.TILES_BATCH])
    k = cache_key(arch, storage, lb.TILES_BATCH, box_class(timer.sites // len(jobs)))
    cache[k] = {"ty": best[0], "tz": best[1], "ms": round(best[2], 4), "jobs": len(jobs),
                "sites": timer.sites, "timings": res}
    log("%s: ty %d tz %d %.4f ms per step" % (k, best[0], best[1], best[2]))
    return {k: cache[k]}


def main():
    ap = argparse.ArgumentParser(description="time tile shapes and cache the fastest")
    ap.add_argument("--n", type=int, default=128, help="side of the emulsion lattice")
    ap.add_argument("--storage", default="f32,f16", help="storages of the single-lattice kinds")
    ap.add_argument("--batch", default="f16", help="storages of the batched step ('' = skip)")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--out", default=os.environ.get("LB_TILE_CACHE", "tiles.json"))
    args = ap.parse_args()
    codes = {v: k for k, v in STORAGE_NAME.items()}
    import torch
    torch.cuda.set_device(0)
    arch = device_arch()
    cache = load(args.out)
    for name in filter(None, args.storage.split(",")):
        tune_lattice(args.n, codes[name], arch, cache, args.steps)
    for name in filter(None, args.batch.split(",")):
        tune_batch(codes[name], arch, cache)
    save(cache, args.out)
    print(json.dumps({k: {kk: v[kk] for kk in ("ty", "tz", "ms")} for k, v in cache.items()}), flush=True)


if __name__ == "__main__":
    main()

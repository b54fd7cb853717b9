"""Continuous-batching serving loop for design-sweep jobs.

Requests (a lattice's parameters plus its emulsion's droplet list and a step
count) arrive over time.  At every chunk edge the server

1. admits waiting requests in arrival order while a slot and arena (HBM
   budget) space are free -- a request that does not fit waits and later ones
   may pass it (backfill); a request larger than the whole budget is rejected;
2. advances every admitted job by one chunk of steps on the device, in one
   batched step per step (a captured graph of `chunk` steps);
3. completes jobs that have taken their steps: it reads their compensated
   totals to the host, flags a job whose state went non-finite (the others
   are unaffected), frees its slot and memory and records its latency
   (arrival -> results on the host).

Jobs admitted while others are mid-run share the device with them: the batch
steps all of them together.  The backend interface is small so that the
scheduling logic is testable without a GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import workloads as W


@dataclass
class Request:
    job_id: int
    arrival: float            # seconds after the stream starts
    params: dict
    centres: np.ndarray
    radii: np.ndarray
    steps: int

    @property
    def sites(self) -> int:
        return int(self.params["nx"]) * int(self.params["ny"]) * int(self.params["nz"])


@dataclass
class Outcome:
    job_id: int
    status: str               # "done", "failed" (non-finite state) or "rejected"
    arrival: float
    admitted: Optional[float] = None
    finished: Optional[float] = None
    sites: int = 0
    steps: int = 0
    totals: Optional[list] = None
    error: str = ""

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class GpuBackend:
    """The library's batched step (lb_batch_*): one arena = the HBM budget."""

    def __init__(self, budget_bytes: int, max_jobs: int = 256, storage: int = W.F16,
                 chunk: int = 50, stream=None):
        from . import lb
        self.lb = lb
        self.batch = lb.Batch(max_jobs, budget_bytes, storage, chunk, stream)
        self.storage = storage
        self.max_jobs = max_jobs
        self.budget = budget_bytes

    def job_bytes(self, params: dict) -> int:
        return self.lb.lb_batch_job_bytes(dict(params, storage=self.storage))

    def admit(self, req: Request) -> Optional[int]:
        try:
            return self.batch.add_droplets(req.params, req.centres, req.radii, req.steps)
        except self.lb.LbError as e:
            if e.code == self.lb.LB_ENOMEM:
                return None
            raise

    def advance(self, n: int) -> None:
        import torch
        self.batch.step(n)
        torch.cuda.synchronize()

    def steps_done(self, slot: int) -> int:
        return self.batch.job_steps(slot)

    def collect(self, slot: int) -> np.ndarray:
        return self.batch.totals(slot)

    def release(self, slot: int) -> None:
        self.batch.remove(slot)

    def close(self) -> None:
        self.batch.close()


@dataclass
class Report:
    outcomes: List[Outcome]
    makespan: float
    busy: float
    chunks: int
    peak_active: int

    def summary(self) -> dict:
        done = [o for o in self.outcomes if o.status == "done"]
        lat = np.array([o.latency for o in done]) if done else np.zeros(0)
        work = sum(o.sites * o.steps for o in done)
        return {
            "jobs": len(self.outcomes),
            "done": len(done),
            "failed": sum(o.status == "failed" for o in self.outcomes),
            "rejected": sum(o.status == "rejected" for o in self.outcomes),
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_s": float(lat.mean()) if len(lat) else None,
            "makespan_s": self.makespan,
            "aggregate_mlups": work / self.makespan / 1e6 if self.makespan > 0 else None,
            "device_mlups": work / self.busy / 1e6 if self.busy > 0 else None,
            "chunks": self.chunks,
            "peak_active": self.peak_active,
        }


class Server:
    def __init__(self, backend, chunk: int = 50, clock=time.perf_counter, sleep=time.sleep):
        self.backend = backend
        self.chunk = int(chunk)
        self.clock = clock
        self.sleep = sleep

    def run(self, requests: List[Request], log=None) -> Report:
        reqs = sorted(requests, key=lambda r: r.arrival)
        outcomes: Dict[int, Outcome] = {}
        waiting: deque = deque()
        active: Dict[int, Request] = {}
        nxt = 0
        busy = 0.0
        chunks = 0
        peak = 0
        budget = getattr(self.backend, "budget", None)
        t0 = self.clock()
        while nxt < len(reqs) or waiting or active:
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                outcomes[r.job_id] = Outcome(r.job_id, "waiting", r.arrival, sites=r.sites,
                                             steps=r.steps)
                waiting.append(r)
                nxt += 1
            # admission in arrival order, with backfill
            for r in list(waiting):
                if len(active) >= self.backend.max_jobs:
                    break
                try:
                    need = self.backend.job_bytes(r.params)
                except Exception as e:      # invalid parameters
                    need = -1
                if need < 0 or (budget is not None and need > budget):
                    o = outcomes[r.job_id]
                    o.status, o.error = "rejected", "invalid parameters or larger than the budget"
                    waiting.remove(r)
                    continue
                try:
                    slot = self.backend.admit(r)
                except Exception as e:
                    o = outcomes[r.job_id]
                    o.status, o.error = "rejected", str(e)
                    waiting.remove(r)
                    continue
                if slot is None:
                    continue
                waiting.remove(r)
                active[slot] = r
                outcomes[r.job_id].admitted = self.clock() - t0
                outcomes[r.job_id].status = "running"
            peak = max(peak, len(active))
            if not active:
                if nxt < len(reqs):
                    wait = reqs[nxt].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                    continue
                if waiting:
                    # nothing runs and nothing fits: reject what is left
                    for r in waiting:
                        outcomes[r.job_id].status = "rejected"
                        outcomes[r.job_id].error = "never fits the budget"
                    waiting.clear()
                break
            t1 = self.clock()
            self.backend.advance(self.chunk)
            busy += self.clock() - t1
            chunks += 1
            now = self.clock() - t0
            for slot in list(active):
                r = active[slot]
                if self.backend.steps_done(slot) >= r.steps:
                    tot = self.backend.collect(slot)
                    o = outcomes[r.job_id]
                    o.finished = self.clock() - t0
                    o.totals = np.asarray(tot).tolist()
                    bad = float(tot[6][0] + tot[6][1]) if tot is not None else 1.0
                    finite = tot is not None and np.all(np.isfinite(tot))
                    o.status = "done" if (finite and bad == 0.0) else "failed"
                    if o.status == "failed":
                        o.error = "non-finite or non-positive density"
                    self.backend.release(slot)
                    del active[slot]
            if log is not None and chunks % 20 == 0:
                log("t=%.1fs chunks=%d active=%d waiting=%d done=%d" % (
                    now, chunks, len(active), len(waiting),
                    sum(o.status in ("done", "failed") for o in outcomes.values())))
        end = self.clock() - t0
        first = reqs[0].arrival if reqs else 0.0
        return Report(list(outcomes.values()), end - first, busy, chunks, peak)


def make_requests(n_jobs: int, seed: int = 0, rate: float = 40.0, steps: int = 500, workers: int = 16,
                  sides=(32, 48, 64, 96, 128)) -> List[Request]:
    """The design-sweep request stream: Poisson arrivals, per-job parameters
    and droplet lists (built by the client, in parallel worker processes; call
    it before the calling process initialises the GPU)."""
    jobs = W.job_stream(seed=seed, n_jobs=n_jobs, rate=rate, sides=sides, steps=steps)
    if workers > 1 and n_jobs > 1:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ctx.Pool(min(workers, n_jobs)) as pool:
            lists = pool.map(_droplets_of, jobs, chunksize=4)
    else:
        lists = [_droplets_of(j) for j in jobs]
    out = []
    for j, (c, r) in zip(jobs, lists):
        out.append(Request(j.job_id, j.arrival, j.params(W.F16), c, r, j.steps))
    return out


def _droplets_of(job):
    c, r, _ = job.droplets()
    return np.asarray(c, dtype=np.float64), np.asarray(r, dtype=np.float64)


def main():
    ap = argparse.ArgumentParser(description="serve a stream of design-sweep jobs on one GPU")
    ap.add_argument("--jobs", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=40.0)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--budget-gb", type=float, default=0.8 * 288)
    ap.add_argument("--max-jobs", type=int, default=512)
    ap.add_argument("--storage", default="f16")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    storage = {"f32": W.F32, "f16": W.F16, "bf16": W.BF16}[args.storage]
    # requests are built by worker processes before this process touches the GPU
    t = time.perf_counter()
    reqs = make_requests(args.jobs, seed=args.seed, rate=args.rate, steps=args.steps)
    for r in reqs:
        r.params = dict(r.params, storage=storage)
    print("[serve] %d requests prepared in %.1fs" % (len(reqs), time.perf_counter() - t), flush=True)
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    backend = GpuBackend(int(args.budget_gb * 2 ** 30), args.max_jobs, storage, args.chunk, stream)
    with torch.cuda.stream(stream):
        rep = Server(backend, args.chunk).run(reqs, log=lambda m: print("[serve] " + m, flush=True))
    backend.close()
    print(json.dumps(rep.summary()), flush=True)


if __name__ == "__main__":
    main()

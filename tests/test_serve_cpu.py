"""Scheduling logic of the serving loop, on a fake device backend (no GPU):
admission by budget and slots, continuous batching, latency accounting,
rejection and failure isolation."""
import numpy as np
import pytest

from paper_2005_12764_amd import serve as S
from paper_2005_12764_amd import workloads as W


class FakeBackend:
    """Slots and an arena budget like the batched step; a chunk of n steps
    takes n * sites * 1e-9 simulated seconds of device time."""

    def __init__(self, budget, max_jobs=4, poison=()):
        self.budget = budget
        self.max_jobs = max_jobs
        self.used = 0
        self.jobs = {}
        self.poison = set(poison)
        self.now = 0.0
        self.peak_used = 0
        self.history = []

    def clock(self):
        return self.now

    def sleep(self, dt):
        self.now += dt

    def job_bytes(self, params):
        if params["tau_r"] <= 0.5:
            raise ValueError("bad tau")
        return 70 * 2 * params["nx"] * params["ny"] * params["nz"]

    def admit(self, req):
        b = self.job_bytes(req.params)
        if len(self.jobs) >= self.max_jobs or self.used + b > self.budget:
            return None
        slot = min(set(range(self.max_jobs)) - set(self.jobs))
        self.jobs[slot] = dict(req=req, done=0, bytes=b)
        self.used += b
        self.peak_used = max(self.peak_used, self.used)
        return slot

    def advance(self, n):
        work = 0
        for j in self.jobs.values():
            k = min(n, j["req"].steps - j["done"])
            j["done"] += k
            work += k * j["req"].sites
        self.history.append(len(self.jobs))
        self.now += work * 1e-9 + 1e-4

    def steps_done(self, slot):
        return self.jobs[slot]["done"]

    def collect(self, slot):
        t = np.zeros((7, 2))
        r = self.jobs[slot]["req"]
        t[0, 0] = r.sites
        if r.job_id in self.poison:
            t[0, 0] = np.nan
            t[6, 0] = 1.0
        return t

    def release(self, slot):
        self.used -= self.jobs.pop(slot)["bytes"]


def _requests(n, rate=40.0, steps=100, side=32, seed=0):
    jobs = W.job_stream(seed=seed, n_jobs=n, rate=rate, sides=(side,), steps=steps)
    return [S.Request(j.job_id, j.arrival, j.params(W.F16), np.zeros((0, 3)), np.zeros(0), steps)
            for j in jobs]


def test_all_jobs_complete_with_latency_accounting():
    fb = FakeBackend(budget=10 * 70 * 2 * 32 ** 3, max_jobs=8)
    reqs = _requests(30)
    rep = S.Server(fb, chunk=20, clock=fb.clock, sleep=fb.sleep).run(reqs)
    s = rep.summary()
    assert s["done"] == 30 and s["failed"] == 0 and s["rejected"] == 0
    for o in rep.outcomes:
        assert o.admitted >= o.arrival - 1e-12 and o.finished > o.admitted
        assert o.latency >= 100 * 32 ** 3 * 1e-9 * 0.99      # at least its own service time
    assert s["p99_s"] >= s["p50_s"] > 0


def test_admission_respects_budget_and_slots():
    budget = 3 * 70 * 2 * 32 ** 3
    fb = FakeBackend(budget=budget, max_jobs=8)
    rep = S.Server(fb, chunk=10, clock=fb.clock, sleep=fb.sleep).run(_requests(20, rate=1e4))
    assert fb.peak_used <= budget
    assert max(fb.history) <= 3                      # the budget, not the slots, binds
    assert rep.summary()["done"] == 20


def test_continuous_batching_admits_arrivals_mid_run():
    fb = FakeBackend(budget=10 ** 12, max_jobs=16)
    reqs = _requests(10, rate=400.0, steps=400)      # arrivals every ~2.5 ms, jobs ~13 ms
    rep = S.Server(fb, chunk=20, clock=fb.clock, sleep=fb.sleep).run(reqs)
    assert rep.peak_active > 1
    # some job was admitted while an earlier one was still running
    outs = sorted(rep.outcomes, key=lambda o: o.arrival)
    assert any(b.admitted < a.finished for a, b in zip(outs, outs[1:]))


def test_failed_job_is_isolated():
    fb = FakeBackend(budget=10 ** 12, max_jobs=8, poison={3})
    rep = S.Server(fb, chunk=25, clock=fb.clock, sleep=fb.sleep).run(_requests(8))
    st = {o.job_id: o.status for o in rep.outcomes}
    assert st[3] == "failed"
    assert all(v == "done" for k, v in st.items() if k != 3)


def test_oversized_and_invalid_jobs_are_rejected():
    fb = FakeBackend(budget=2 * 70 * 2 * 32 ** 3, max_jobs=4)
    reqs = _requests(6)
    big = W.base_params(64, 64, 64, storage=W.F16, tau_r=0.8, tau_b=0.8)
    bad = W.base_params(32, 32, 32, storage=W.F16, tau_r=0.4, tau_b=0.8)
    reqs.append(S.Request(100, 0.01, big, np.zeros((0, 3)), np.zeros(0), 50))
    reqs.append(S.Request(101, 0.02, bad, np.zeros((0, 3)), np.zeros(0), 50))
    rep = S.Server(fb, chunk=25, clock=fb.clock, sleep=fb.sleep).run(reqs)
    st = {o.job_id: o.status for o in rep.outcomes}
    assert st[100] == "rejected" and st[101] == "rejected"
    assert sum(v == "done" for v in st.values()) == 6

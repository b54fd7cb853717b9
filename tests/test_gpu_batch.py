"""GPU tests of the batched step, the droplet initialiser and the serving loop.

- a job's result is bitwise the same alone in a batch, in a mix of uneven jobs,
  and as a single lattice stepped by the one-read step on the same tile boxes
  (8 rows, 32-plane chunks); and matches the oracle (FP32) within 1e-5;
- jobs stop at their own step counts; graph replays equal eager steps;
- the arena enforces the HBM budget and is reused after removal;
- the droplet initialiser reproduces the host generator's fields;
- the serving loop completes a short request stream, each result equal to the
  same job run alone.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_12764_amd import lb
from paper_2005_12764_amd import serve as S
from paper_2005_12764_amd import workloads as W
from tests.helpers import oracle_params, state_errors

pytestmark = pytest.mark.gpu

# the batch's default tile boxes: 8-row tiles, 32-plane chunks
BATCH_TY, BATCH_TZ = 8, 32


def single_one_read(params, rr, rb, steps):
    """The job as a single lattice, one-read step on the batch's tile boxes."""
    st = params["storage"]
    lb.lb_set_tiles(lb.TILES_ONE_READ, st, BATCH_TY, BATCH_TZ)
    try:
        with lb.Lattice(dict(params, kernel=lb.KERNEL_FUSED)) as L:
            L.init(rr, rb).step(steps)
            return L.state()
    finally:
        lb.lb_set_tiles(lb.TILES_ONE_READ, st, 0, 0)


def _jobs(storage):
    a = W.two_droplets(n=(48, 24, 20), R=6, gap=2.0, A=0.01, nc_strength=0.03, nc_range=2,
                       storage=storage)
    a.params["tau_r"], a.params["tau_b"] = 0.8, 1.1
    b = W.single_droplet(seed=1, n=32, R=7, storage=storage)
    c = W.crystal_channel(seed=3, nx=70, ny=40, nz=22, R=6, spacing=14, storage=storage)
    return a, b, c


@pytest.mark.parametrize("storage", [W.F32, W.F16])
def test_job_alone_equals_job_in_mix_and_single_lattice(storage):
    a, b, c = _jobs(storage)
    steps = 60
    with lb.Batch(8, 1 << 30, storage, graph_steps=20) as B:
        sa = B.add(a.params, a.rho_r, a.rho_b, steps=steps)
        B.step(steps)
        alone = B.state(sa)
    with lb.Batch(8, 1 << 30, storage, graph_steps=20) as B:
        sb = B.add(b.params, b.rho_r, b.rho_b, steps=steps + 7)
        B.step(5)                                   # b is mid-run when a arrives
        sa = B.add(a.params, a.rho_r, a.rho_b, steps=steps)
        sc = B.add(c.params, c.rho_r, c.rho_b, steps=steps)
        B.step(steps + 10)
        mixed = B.state(sa)
        assert B.job_steps(sa) == steps and B.job_steps(sc) == steps and B.job_steps(sb) == steps + 7
    assert np.array_equal(alone, mixed)
    # the batch runs the single lattice's one-read tile code on the same tile
    # boxes: bitwise equal; the two-pass step gathers phi in another order of
    # summation, so it agrees to rounding
    single = single_one_read(dict(a.params, storage=storage), a.rho_r, a.rho_b, steps)
    assert np.array_equal(alone, single)
    with lb.Lattice(dict(a.params, storage=storage, kernel=lb.KERNEL_TWOPASS)) as L:
        L.init(a.rho_r, a.rho_b).step(steps)
        two = L.state()
    assert state_errors(two, alone)["worst"] < (1e-6 if storage == W.F32 else 1e-3)
    for job in (b, c):
        with lb.Batch(8, 1 << 30, storage, graph_steps=20) as B:
            sl = B.add(job.params, job.rho_r, job.rho_b, steps=steps)
            B.step(steps)
            got = B.state(sl)
        assert np.array_equal(got, single_one_read(dict(job.params, storage=storage), job.rho_r, job.rho_b,
                                                   steps)), job.name
    if storage == W.F32:
        ref = O.step(oracle_params(a.params), O.init(oracle_params(a.params), a.rho_r, a.rho_b), steps)
        assert state_errors(mixed, ref)["worst"] < 1e-5


def test_graph_replay_equals_eager_steps():
    a, b, _ = _jobs(W.F32)
    with lb.Batch(4, 1 << 28, W.F32, graph_steps=8) as G, lb.Batch(4, 1 << 28, W.F32, graph_steps=8) as E:
        ga = G.add(a.params, a.rho_r, a.rho_b, steps=100)
        ea = E.add(a.params, a.rho_r, a.rho_b, steps=100)
        G.step(8 * 5 + 3)                            # 5 replays + 3 eager steps
        for _ in range(43):
            E.step(1)
        assert np.array_equal(G.state(ga), E.state(ea))


def test_arena_budget_and_reuse():
    p = W.base_params(64, 64, 64, storage=W.F16, tau_r=0.9, tau_b=0.9, A=0.01)
    jb = lb.lb_batch_job_bytes(p)
    assert jb >= 2 * 70 * 64 ** 3
    rr = np.full((64, 64, 64), 0.5)
    with lb.Batch(8, 2 * jb + 4096, W.F16, graph_steps=4) as B:
        s1 = B.add(p, rr, rr, steps=10)
        s2 = B.add(p, rr, rr, steps=10)
        with pytest.raises(lb.LbError) as e:
            B.add(p, rr, rr, steps=10)
        assert e.value.code == lb.LB_ENOMEM
        B.step(4)
        B.remove(s1)
        s3 = B.add(p, rr, rr, steps=10)             # the freed space is reused
        B.step(12)
        assert B.job_steps(s3) == 10 and B.job_steps(s2) == 10
        t = B.totals(s3)
        assert abs(t[0].sum() / (0.5 * 64 ** 3) - 1) < 1e-6


def test_droplet_initialiser_matches_host_fields():
    rng = np.random.default_rng(5)
    n = (40, 36, 28)
    cen, rad, _ = W.emulsion(rng, n, 0.25, 5.0, 8.0)
    for bc in ((0, 0, 0), (0, 1, 1)):
        phi = W.droplet_phase(n[::-1], cen, rad, bc=bc)
        rr, rb = W.split_components(phi, 1.0)
        p = W.base_params(*n, bc=bc, storage=W.F64, tau_r=0.9, tau_b=0.9)
        with lb.Lattice(p) as A, lb.Lattice(p) as B:
            A.init(rr, rb)
            B.init_droplets(cen, rad)
            fa, fb = A.state(), B.state()
        assert np.abs(fa - fb).max() < 1e-14


def test_serving_loop_short_stream():
    import torch
    reqs = S.make_requests(10, seed=3, rate=200.0, steps=60, workers=1, sides=(32, 48))
    stream = torch.cuda.Stream()
    be = S.GpuBackend(1 << 30, max_jobs=6, storage=W.F16, chunk=20, stream=stream)
    with torch.cuda.stream(stream):
        rep = S.Server(be, chunk=20).run(reqs)
    be.close()
    s = rep.summary()
    assert s["done"] == 10 and s["failed"] == 0 and rep.peak_active > 1
    # each job's totals equal the same job run alone
    for o in rep.outcomes[:3]:
        r = next(q for q in reqs if q.job_id == o.job_id)
        with lb.Batch(2, 1 << 28, W.F16, graph_steps=20) as B:
            sl = B.add_droplets(r.params, r.centres, r.radii, r.steps)
            B.step(r.steps)
            alone = B.totals(sl)
        assert np.array_equal(np.asarray(o.totals), alone)


def test_f16_job_with_its_own_scale_matches_single_lattice():
    # a batched fp16 job steps with its own deviation scale 2^scale_log2, as a
    # single lattice with the same parameters does (bitwise: same tile code)
    _, b, _ = _jobs(W.F16)
    for s2 in (12, 20):
        p = dict(b.params, storage=W.F16, scale_log2=s2)
        with lb.Batch(2, 1 << 28, W.F16, graph_steps=10) as B:
            sl = B.add(p, b.rho_r, b.rho_b, steps=30)
            B.step(30)
            batched = B.state(sl)
        assert np.array_equal(batched, single_one_read(p, b.rho_r, b.rho_b, 30)), s2


def test_zero_step_16bit_job_is_rejected():
    _, b, _ = _jobs(W.F16)
    with lb.Batch(2, 1 << 28, W.F16, graph_steps=10) as B:
        with pytest.raises(lb.LbError) as e:
            B.add(b.params, b.rho_r, b.rho_b, steps=0)
        assert e.value.code == lb.LB_EINVAL
        assert B.free_bytes() == 1 << 28
    with lb.Batch(2, 1 << 28, W.F32, graph_steps=10) as B:
        p = dict(b.params, storage=W.F32)
        sl = B.add(p, b.rho_r, b.rho_b, steps=0)     # raw storage keeps its initial state
        f = B.state(sl)
        with lb.Lattice(p) as L:
            L.init(b.rho_r, b.rho_b)
            assert np.array_equal(f, L.state())


@pytest.mark.parametrize("storage", [W.F64, W.BF16])
def test_four_row_tiles_and_short_chunks_match_single_lattice(storage):
    # the batch's other tile rows (4) with 16-plane chunks: ragged x tiles,
    # walls and a chunk shorter than the rest, bitwise the single lattice's
    # one-read step on the same boxes
    _, _, c = _jobs(storage)
    p = dict(c.params, storage=storage)
    lb.lb_set_tiles(lb.TILES_BATCH, storage, 4, 16)
    try:
        with lb.Batch(2, 1 << 29, storage, graph_steps=10) as B:
            sl = B.add(p, c.rho_r, c.rho_b, steps=25)
            B.step(25)
            got = B.state(sl)
    finally:
        lb.lb_set_tiles(lb.TILES_BATCH, storage, 0, 0)
    lb.lb_set_tiles(lb.TILES_ONE_READ, storage, 4, 16)
    try:
        with lb.Lattice(dict(p, kernel=lb.KERNEL_FUSED)) as L:
            L.init(c.rho_r, c.rho_b).step(25)
            single = L.state()
    finally:
        lb.lb_set_tiles(lb.TILES_ONE_READ, storage, 0, 0)
    assert np.array_equal(got, single)

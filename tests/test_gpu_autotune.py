"""Tile shapes on the GPU: results independent of the shape where the method
fixes them (two-pass steps), following the tile boxes where the phase sums
do (one-read and batched steps), the one-read step safe across a change of
shape, the tuner's choices runnable."""
import numpy as np
import pytest

from paper_2005_12764_amd import autotune as T
from paper_2005_12764_amd import lb
from paper_2005_12764_amd import workloads as W
from tests.helpers import state_errors

pytestmark = pytest.mark.gpu


@pytest.fixture
def tiles():
    """lb_set_tiles for the test, every setting cleared afterwards."""
    yield lb.lb_set_tiles
    for kind in (lb.TILES_PHASE, lb.TILES_COLLIDE, lb.TILES_ONE_READ, lb.TILES_BATCH):
        for st in (W.F64, W.F32, W.F16, W.BF16):
            lb.lb_set_tiles(kind, st, 0, 0)


def _run(w, storage, kernel, steps):
    with lb.Lattice(dict(w.params, storage=storage, kernel=kernel)) as L:
        L.init(w.rho_r, w.rho_b).step(steps)
        return L.state()


@pytest.mark.parametrize("storage", [W.F32, W.F16])
def test_two_pass_results_do_not_depend_on_tiles(storage, tiles):
    w = W.two_droplets(n=(70, 21, 19), R=6, gap=2.0, A=0.01, nc_strength=0.03, nc_range=2)
    a = _run(w, storage, lb.KERNEL_TWOPASS, 12)
    tiles(lb.TILES_COLLIDE, storage, 2, 5)
    tiles(lb.TILES_PHASE, storage, 16, 3)
    b = _run(w, storage, lb.KERNEL_TWOPASS, 12)
    assert np.array_equal(a, b)


def test_one_read_survives_a_change_of_tiles(tiles):
    w = W.two_droplets(n=(70, 21, 19), R=6, gap=2.0, A=0.01, nc_strength=0.03, nc_range=2)
    ref = _run(w, W.F64, lb.KERNEL_TWOPASS, 20)
    with lb.Lattice(dict(w.params, storage=W.F64, kernel=lb.KERNEL_FUSED)) as L:
        L.init(w.rho_r, w.rho_b).step(10)
        tiles(lb.TILES_ONE_READ, W.F64, 4, 6)   # the sums of the old boxes are not reused
        L.step(10)
        assert L.kernel == lb.KERNEL_FUSED
        got = L.state()
    assert state_errors(got, ref)["worst"] < 1e-13


def test_one_read_with_sixteen_rows(tiles):
    # 1024-thread tiles: agree with the two-pass step to FP32 rounding and
    # resume from a checkpoint bit for bit
    w = W.two_droplets(n=(70, 40, 19), R=6, gap=2.0, A=0.01, nc_strength=0.03, nc_range=2)
    w.params["bc"] = (0, 1, 0)
    ref = _run(w, W.F32, lb.KERNEL_TWOPASS, 30)
    tiles(lb.TILES_ONE_READ, W.F32, 16, 0)
    p = dict(w.params, storage=W.F32, kernel=lb.KERNEL_FUSED)
    with lb.Lattice(p) as A, lb.Lattice(p) as B:
        A.init(w.rho_r, w.rho_b).step(12)
        ck = A.save_raw()
        A.step(18)
        straight = A.state()
        B.init(w.rho_r, w.rho_b).step(1)
        B.load_raw(ck)
        B.step(18)
        assert np.array_equal(B.state(), straight)
    assert state_errors(straight, ref)["worst"] < 2e-6


def test_batch_results_follow_their_tile_boxes(tiles):
    # the batched step is the one-read step on the batch's tile boxes: other
    # boxes move the results by rounding only, and each shape equals the
    # single lattice's one-read step on the same boxes bitwise
    jobs = [W.periodic_emulsion(seed=k, n=s) for k, s in enumerate((32, 48))]

    def run():
        with lb.Batch(4, 1 << 30, W.F16, graph_steps=10) as B:
            slots = [B.add(dict(w.params, storage=W.F16), w.rho_r, w.rho_b, steps=20) for w in jobs]
            B.step(20)
            return [B.state(s) for s in slots]

    def single(w, ty, tz):
        tiles(lb.TILES_ONE_READ, W.F16, ty, tz)
        return _run(w, W.F16, lb.KERNEL_FUSED, 20)

    a = run()
    tiles(lb.TILES_BATCH, W.F16, 4, 16)
    b = run()
    for w, x, y in zip(jobs, a, b):
        assert state_errors(x, y)["worst"] < 1e-3
        assert np.array_equal(x, single(w, 8, 32))
        assert np.array_equal(y, single(w, 4, 16))


def test_tuner_picks_runnable_shapes(tmp_path, tiles):
    cache = {}
    arch = T.device_arch()
    out = T.tune_lattice(32, W.F32, arch, cache, steps=4, log=lambda m: print(m, flush=True))
    out.update(T.tune_batch(W.F16, arch, cache, sides=(32,), copies=2, steps=4,
                            log=lambda m: print(m, flush=True)))
    assert set(out) == {T.cache_key(arch, W.F32, lb.TILES_ONE_READ, "small"),
                        T.cache_key(arch, W.F32, lb.TILES_COLLIDE, "small"),
                        T.cache_key(arch, W.F16, lb.TILES_BATCH, "small")}
    for e in out.values():
        assert (e["ty"], e["tz"]) in [(r["ty"], r["tz"]) for r in e["timings"] if r["ms"] is not None]
    path = str(tmp_path / "tiles.json")
    T.save(cache, path)
    assert T.apply(T.load(path), arch, W.F32, 32 ** 3)
    w = W.periodic_emulsion(seed=0, n=32)
    assert np.isfinite(_run(w, W.F32, lb.KERNEL_AUTO, 4)).all()

"""The one-read step's memory access pattern without arithmetic
(lb_pattern_ms), the bench's ceiling for that kernel: it runs on its own
buffers and stream, leaves a lattice's state alone, and takes no longer than
the step's own tile kernel does with its arithmetic."""
import numpy as np
import pytest

from paper_2005_12764_amd import lb
from paper_2005_12764_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_pattern_runs_beside_a_lattice_without_touching_it():
    w = W.periodic_emulsion(seed=0, n=64, storage=W.F32)
    with lb.Lattice(w.params) as L:
        L.init(w.rho_r, w.rho_b).step(3)
        f0 = L.state()
        ms = lb.lb_pattern_ms(w.params, 5)
        assert np.isfinite(ms) and 0.0 < ms < 50.0
        assert np.array_equal(L.state(), f0)
        L.step(1)
        assert np.isfinite(L.state()).all()


def test_pattern_is_a_ceiling_for_the_one_read_tile():
    # 128^3 periodic emulsion: the step's tile kernel (with its arithmetic)
    # takes at least as long as the same access pattern without it
    w = W.periodic_emulsion(seed=0, n=128, storage=W.F32)
    with lb.Lattice(w.params) as L:
        L.init(w.rho_r, w.rho_b).step(2)
        assert L.kernel == lb.KERNEL_FUSED
        tile_ms = min(lb.lb_step_timed(L.h, 5)[1] for _ in range(3))
    pat_ms = min(lb.lb_pattern_ms(w.params, 10) for _ in range(3))
    print("128^3: tile %.3f ms, access pattern alone %.3f ms" % (tile_ms, pat_ms), flush=True)
    assert pat_ms <= 1.05 * tile_ms

"""The benchmark set-ups as committed checks (GPU):

- spinodal decomposition (the arrested-coarsening bijel of the LBsoft section,
  384^3 in the benchmark): FP32 against the oracle pointwise over its early,
  still deterministic steps; the 16-bit forms against FP32 by the structure
  factor (first moment k1 and peak height) once domains have formed;
- the microfluidic-crystal channel (512x128x64, walls in y and z, body force,
  near contact) over its full 2000 steps: FP32 and the 16-bit forms against
  the FP64 run with the same |G| threshold;
- steady flow in the channel's 128x64 cross-section against the duct's
  Fourier series.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_12764_amd import lb
from paper_2005_12764_amd import workloads as W
from tests.helpers import duct_series, oracle_params, state_errors, structure_factor

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("steps", [10, 25])
def test_spinodal_f32_matches_the_oracle_early(steps):
    # before interfaces form |G| stays below the near-contact threshold and
    # far above eps_G, so no decision can flip: the FP32 bound holds
    # pointwise (later steps are covered one step at a time, with the
    # threshold sites located, in test_gpu_fp32_flips.py)
    w = W.spinodal(seed=0, n=64, storage=W.F32)
    with lb.Lattice(w.params) as L:
        L.init(w.rho_r, w.rho_b).step(steps)
        f = L.state()
    prm = oracle_params(w.params)
    ref = O.step(prm, O.init(prm, w.rho_r, w.rho_b), steps)
    e = state_errors(f, ref)
    print("spinodal 64^3 %d steps f32 vs oracle: %s" % (steps, e), flush=True)
    assert e["worst"] <= 1e-5


def test_spinodal_16bit_structure_factor_tracks_fp32():
    w = W.spinodal(seed=0, n=128)
    out = {}
    for storage in (W.F32, W.F16, W.BF16):
        with lb.Lattice(dict(w.params, storage=storage)) as L:
            L.init(w.rho_r, w.rho_b)
            out[storage] = []
            for _ in range(2):
                L.step(300)
                rr, rb, _ = L.moments()
                out[storage].append(structure_factor((rr - rb) / (rr + rb)))
    for storage in (W.F16, W.BF16):
        for (k1, peak), (k1r, peakr) in zip(out[storage], out[W.F32]):
            print("spinodal 128^3 storage=%d k1 %.4f (f32 %.4f) peak %.4e (f32 %.4e)"
                  % (storage, k1, k1r, peak, peakr), flush=True)
            assert abs(k1 / k1r - 1) <= 0.01
            assert abs(peak / peakr - 1) <= 0.05


def test_crystal_channel_full_length_against_fp64():
    # Over 2000 steps the films between droplets take their own course in
    # each precision: differences start at the |G| -> 0 saddles inside films
    # (the recolouring direction is decided there by the |G| threshold) and a
    # film that thins slightly differently can drain at another step, a local
    # O(0.1) difference.  What must agree is what conservation and the
    # driving fix: each component's mass (exact) and the flow rate.
    w = W.crystal_channel(seed=0)                      # 512x128x64, 2000 steps
    out = {}
    for storage in (W.F64, W.F32, W.F16, W.BF16):
        with lb.Lattice(dict(w.params, storage=storage, eps_g=1e-6)) as L:
            L.init(w.rho_r, w.rho_b)
            t0 = L.totals().sum(1)
            L.step(w.steps)
            out[storage] = (L.totals().sum(1), t0, L.state())
    # (FP32 and 16-bit records round the stored density every step: the masses
    # drift by a random walk of that rounding, ~1e-6 over 2000 steps; the flow
    # rate follows the droplets, which move through the film events, to ~0.4 %)
    ref, _, fref = out[W.F64]
    checks = []
    for storage in (W.F32, W.F16, W.BF16):
        tot, t0, f = out[storage]
        e = state_errors(f, fref)
        flow = tot[2] / ref[2] - 1                    # total x momentum: the flow rate
        dm = max(abs(tot[0] / t0[0] - 1), abs(tot[1] / t0[1] - 1))
        print("crystal channel %d steps storage=%d vs fp64: flow %+.2e, mass drift %.1e, pointwise %s"
              % (w.steps, storage, flow, dm, e), flush=True)
        checks.append((dm, flow, e["worst"]))
    for dm, flow, worst in checks:
        assert dm < 2e-5 and abs(flow) <= 1e-2 and worst <= 5e-2


@pytest.mark.parametrize("storage,tol", [(W.F64, 1e-4), (W.F32, 3e-4), (W.F16, 1e-3), (W.BF16, 5e-3)])
def test_duct_flow_in_the_channel_cross_section(storage, tol):
    a, b, g = 128, 64, 1e-6
    tau = 0.5 + math.sqrt(3) / 4
    nu = (tau - 0.5) / 3
    p = W.base_params(4, a, b, bc=(0, 1, 1), storage=storage, tau_r=tau, tau_b=tau, body_force=(g, 0.0, 0.0))
    rr = np.ones((b, a, 4))
    steps = int(24 * b * b / (nu * math.pi ** 2))      # the slowest mode decays by e^-30
    with lb.Lattice(p) as L:
        L.init(rr, np.zeros_like(rr)).step(steps)
        r1, r2, j = L.moments()
    ux = ((j[0] + g / 2) / (r1 + r2)).mean(axis=2)
    y = np.arange(a) - (a - 1) / 2
    z = np.arange(b) - (b - 1) / 2
    ua = duct_series(a, b, y[None, :], z[:, None], g, nu)
    err = float(np.linalg.norm(ux - ua) / np.linalg.norm(ua))
    print("duct %dx%d storage=%d %d steps: rel L2 %.3e" % (a, b, storage, steps, err), flush=True)
    assert err <= tol

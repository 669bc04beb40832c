"""Kernel plans: every admissible (tile_vpt, cell_lanes) gives the oracle's result, and the
autotuner returns one of them."""
import numpy as np
import pytest

from tests.gpu_helpers import make_pair, parity, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,rounding,tol", [(0, 0, 1e-12), (1, 1, 1e-5)])
def test_every_tiling_matches_the_oracle(precision, rounding, tol):
    # FP32 storage runs the stage kernel's LDS prefetch, whose per-row velocity walk (1 to 12
    # velocities here, the last one loading itself again) each plan exercises
    from paper_1810_07803_amd import hrlb

    Qx, Qy, nx = 8, 12, 100
    say(f"[tiling] Qx={Qx} Qy={Qy} nx={nx} precision={precision}, tile_vpt in divisors of Qy")
    _, orc = make_pair(Qx, Qy, nx, delta=0.7, uw=0.25, stretch_A=0.9)
    phi, chi = orc.init_state()
    orc.step(phi, chi, 12)
    q = hrlb.Quadrature(Qx, Qy)
    for vpt, lanes in ((1, 1), (2, 2), (3, 4), (4, 8), (6, 16), (12, 0)):
        c = hrlb.Case(q, hrlb.make_params(delta=0.7, uw=0.25, ncell=nx, stretch_A=0.9, dt=orc.dt, tile_vpt=vpt,
                                          cell_lanes=lanes, precision=precision, rounding=rounding, seed=3))
        c.step(12)
        say(f"   vpt={vpt} lanes={lanes}")
        assert parity(c.get_state(), phi, chi, c.moments()[0], orc.moments(phi, chi), tol)


def test_autotuner_returns_an_admissible_tiling():
    from paper_1810_07803_amd import hrlb

    say("[tiling] autotuner on nx=512 HHLB(10;16) x HLB(7;8)")
    q = hrlb.Quadrature(16, 8)
    best, lanes, ms = hrlb.tune_plan(q, hrlb.make_params(delta=0.1, uw=0.2, ncell=512, stretch_A=0.9, omega=0.66),
                                     n_steps=5)
    say(f"   best tile_vpt={best} cell_lanes={lanes} at {ms:.4f} ms/step")
    assert best in (1, 2, 4, 8) and lanes in (1, 2, 4, 8, 16) and ms > 0

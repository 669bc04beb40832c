"""Step blocks replayed from captured HIP graphs give bitwise the same states as direct launches,
including replays interleaved with direct launches, residual checks and batches."""
import numpy as np
import pytest

from tests.gpu_helpers import make_pair, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_graph_replays_match_direct_launches(precision, rounding):
    say(f"[graphs] nx128 q8x8 precision={precision}")
    a, _ = make_pair(8, 8, 128, delta=0.5, uw=0.3, stretch_A=0.9, precision=precision, rounding=rounding, seed=3)
    b, _ = make_pair(8, 8, 128, delta=0.5, uw=0.3, stretch_A=0.9, precision=precision, rounding=rounding, seed=3)
    a.set_graph_steps(0)
    b.set_graph_steps(8)
    for n in (37, 8, 3, 16):  # graph blocks, a remainder, direct-only and two replays again
        a.step(n)
        b.step(n)
        np.testing.assert_array_equal(a.get_state(), b.get_state())
    sa, ia = a.run_to_steady(1e-30, 40, 8)
    sb, ib = b.run_to_steady(1e-30, 40, 8)
    assert ia.residual == ib.residual
    np.testing.assert_array_equal(a.moments()[0], b.moments()[0])


def test_batch_graph_replays_match_direct_launches():
    from paper_1810_07803_amd import hrlb

    say("[graphs] batch of 3")
    shapes = [(4, 4, 64), (8, 12, 96), (16, 8, 40)]
    sets = []
    for graph in (0, 5):
        cs = [make_pair(qx, qy, nx, delta=1.0, uw=0.2, precision=1, rounding=1, seed=9)[0] for qx, qy, nx in shapes]
        b = hrlb.Batch(cs)
        b.set_graph_steps(graph)
        b.step(12)
        b.step(10, check=True)
        sets.append((cs, b.poll()))
    for x, y in zip(sets[0][0], sets[1][0]):
        np.testing.assert_array_equal(x.get_state(), y.get_state())
    np.testing.assert_array_equal(sets[0][1][0], sets[1][1][0])


def test_graph_replays_with_local_time_steps_match_direct_launches():
    # checked steps of a local-step case also capture the mass rescaling and the re-analysis
    from paper_1810_07803_amd import hrlb

    say("[graphs] local time steps, checks inside the captured blocks")
    q = hrlb.Quadrature(8, 4)
    kw = dict(delta=0.5, uw=0.4, ncell=64, stretch_A=0.98, half_channel=1, local_dt_cap=32.0, precision=1, rounding=1,
              seed=4)
    a = hrlb.Case(q, hrlb.make_params(**kw))
    b = hrlb.Case(q, hrlb.make_params(**kw))
    a.set_graph_steps(0)
    b.set_graph_steps(10)
    for _ in range(3):  # replays after the program's own work and synchronisations
        sa, ia = a.run_to_steady(1e-300, 40, 10)
        sb, ib = b.run_to_steady(1e-300, 40, 10)
        assert ia.residual == ib.residual and ia.mass_drift == ib.mass_drift
        np.testing.assert_array_equal(a.get_state(), b.get_state())
        np.testing.assert_array_equal(a.moments()[0], b.moments()[0])

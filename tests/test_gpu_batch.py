"""Batched ragged launches: each case's result is bitwise the same alone and in any batch, and the
full-size ragged batch agrees with the oracle on sampled instances."""
import numpy as np
import pytest

from hrlb_inputs import batch_draws
from tests.gpu_helpers import make_pair, parity, say

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 64, 1.0, 0.05), (8, 12, 128, 0.2, 0.3), (16, 8, 100, 5.0, 0.45), (4, 8, 36, 0.02, 0.1)]


def _cases(precision, rounding):
    out = []
    for k, (Qx, Qy, nx, delta, uw) in enumerate(SHAPES):
        c, _ = make_pair(Qx, Qy, nx, delta=delta, uw=uw, stretch_A=0.9, precision=precision, rounding=rounding,
                         seed=100 + k)
        out.append(c)
    return out


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_batch_plan_equals_alone_bitwise(precision, rounding):
    # the benchmark batches' plan (rows of the largest divisor of Q_y up to 16, one lane per cell),
    # requested per case: each case keeps its bits alone and in a batch split over three streams
    import bench
    from paper_1810_07803_amd import hrlb

    def cases():
        out = []
        for k, (Qx, Qy, nx, delta, uw) in enumerate(SHAPES):
            q = hrlb.Quadrature(Qx, Qy)
            c = hrlb.Case(q, hrlb.make_params(delta=delta, uw=uw, ncell=nx, stretch_A=0.9, precision=precision,
                                              rounding=rounding, seed=200 + k, tile_vpt=bench.long_row_vpt(Qx, Qy),
                                              cell_lanes=1))
            c._quad_ref = q
            out.append(c)
        return out

    say(f"[batch] batch plan alone vs mix, precision={precision} rounding={rounding}")
    alone = cases()
    for c in alone:
        c.step(25)
    mixed = cases()
    b = hrlb.Batch(mixed)
    b.set_streams(3)
    b.step(25)
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a.get_state(), m.get_state())
        np.testing.assert_array_equal(a.moments()[0], m.moments()[0])


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_batch_equals_alone_bitwise(precision, rounding):
    from paper_1810_07803_amd import hrlb

    say(f"[batch] alone vs mix, precision={precision} rounding={rounding}, shapes={SHAPES}")
    alone = _cases(precision, rounding)
    for c in alone:
        c.step(25)
    mixed = _cases(precision, rounding)
    b = hrlb.Batch(mixed)
    b.step(25)
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a.get_state(), m.get_state())
        fa, _, pa, _ = a.moments()
        fm, _, pm, _ = m.moments()
        np.testing.assert_array_equal(fa, fm)
    # a different mix (reversed order, one case left out) still gives the same numbers
    again = _cases(precision, rounding)
    b2 = hrlb.Batch(list(reversed(again[1:])))
    b2.step(25)
    for a, m in zip(alone[1:], again[1:]):
        np.testing.assert_array_equal(a.get_state(), m.get_state())


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_batch_split_over_streams_is_bitwise_the_same(precision, rounding):
    from paper_1810_07803_amd import hrlb

    say(f"[batch] 1..4 streams, precision={precision}")
    ref = None
    for n in (1, 2, 3, 4):
        cs = _cases(precision, rounding)
        b = hrlb.Batch(cs)
        b.set_streams(n)
        b.step(12, check=True)
        res, pxy = b.poll()
        states = [c.get_state() for c in cs]
        if ref is None:
            ref = (states, res, pxy)
            continue
        for a, m in zip(ref[0], states):
            np.testing.assert_array_equal(a, m)
        np.testing.assert_array_equal(ref[1], res)
        np.testing.assert_array_equal(ref[2], pxy)


def test_batch_poll_reports_residual_and_pxy():
    from paper_1810_07803_amd import hrlb

    say("[batch] poll")
    cs = _cases(0, 0)
    b = hrlb.Batch(cs)
    b.step(20, check=True)
    res, pxy = b.poll()
    for c, r, p in zip(cs, res, pxy):
        f, x, pi, _ = c.moments()
        assert np.isfinite(r) and r > 0
        jd = np.diff(np.concatenate([[-0.5], 0.5 * (x[1:] + x[:-1]), [0.5]]))  # only a sanity scale
        assert abs(p - np.average(f[5], weights=jd)) < 0.2 * (abs(p) + 1e-6)


@pytest.mark.parametrize("precision,rounding,tol", [(1, 1, 1e-5), (0, 0, 1e-12)])
def test_full_ragged_batch_sampled_against_oracle(precision, rounding, tol):
    """The 512-instance ragged workload (seed 0), launched as one batch in the benchmark's
    configuration (its batch plan: long rows and one lane per cell; three streams); sampled
    instances (the smallest, the median, the largest and one of the 40 largest) are re-run alone by
    the oracle from the rest state with the oracle's own time step, and compared element by element."""
    import bench
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    draws = batch_draws(512, seed=0)
    say(f"[batch] full ragged batch of {len(draws)} instances, precision={precision}")
    cases = []
    for d in draws:
        q = hrlb.Quadrature(d["Qx"], d["Qy"])
        p = hrlb.make_params(delta=d["delta"], uw=d["uw"], ncell=d["ncell"], stretch_A=d["stretch_A"],
                             omega=d["omega"], precision=precision, rounding=rounding, seed=d["seed"],
                             tile_vpt=bench.long_row_vpt(d["Qx"], d["Qy"]), cell_lanes=1)
        c = hrlb.Case(q, p)
        c._quad_ref = q
        cases.append(c)
    b = hrlb.Batch(cases)
    steps = 3
    b.step(steps)
    sizes = [d["ncell"] * 2 * d["Qx"] * d["Qy"] for d in draws]
    order = np.argsort(sizes)
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-20]), int(order[-1])]
    ok = True
    for k in sample:
        d = draws[k]
        say(f"   sample {k}: {d}")
        orc = OracleProblem(d["Qx"], d["Qy"], d["ncell"], delta=d["delta"], uw=d["uw"], stretch_A=d["stretch_A"],
                            omega=d["omega"])
        assert orc.dt == pytest.approx(cases[k].dt, rel=1e-14)
        phi, chi = orc.init_state()
        orc.step(phi, chi, steps)
        ok = parity(cases[k].get_state(), phi, chi, cases[k].moments()[0], orc.moments(phi, chi), tol) and ok
    assert ok

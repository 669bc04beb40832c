"""Time averages of the fields (hrlb_average_*): the running sums kept by the per-cell kernel equal
the mean of the per-step moments read back one step at a time, alone and inside a batch, on the
small-case path over multi-step launches, and stop when asked."""
import numpy as np
import pytest

from tests.gpu_helpers import make_pair, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_average_equals_mean_of_step_moments(precision):
    say(f"[average] nx64 q8x4 precision={precision}")
    case, _ = make_pair(8, 4, 64, delta=1.0, uw=0.2, stretch_A=0.9, precision=precision, rounding=precision)
    case.step(10)
    case.average_start()
    acc = np.zeros((10, 64))
    for _ in range(7):
        case.step(1)
        f, _, _, _ = case.moments()
        acc += f
    fa, pi, n = case.average_read()
    assert n == 7
    np.testing.assert_allclose(fa, acc / 7, rtol=1e-14, atol=1e-15)
    case.average_stop()
    case.step(3)
    fb, _, n2 = case.average_read()
    assert n2 == 7
    np.testing.assert_array_equal(fa, fb)


def test_average_inside_a_batch():
    from paper_1810_07803_amd import hrlb

    say("[average] two cases in a batch, one averaged")
    a, _ = make_pair(4, 4, 32, delta=1.0, uw=0.05)
    b, _ = make_pair(8, 8, 64, delta=0.3, uw=0.3, stretch_A=0.9)
    batch = hrlb.Batch([a, b])
    batch.step(5)
    b.average_start()
    acc = np.zeros((10, 64))
    for _ in range(4):
        batch.step(1)
        f, _, _, _ = b.moments()
        acc += f
    fb, _, n = b.average_read()
    assert n == 4
    np.testing.assert_allclose(fb, acc / 4, rtol=1e-14, atol=1e-15)
    with pytest.raises(hrlb.HrlbError):
        a.average_read()


@pytest.mark.parametrize("precision", [0, 1])
def test_average_on_the_small_case_path(precision):
    # the small-case kernel runs a block of steps per launch and keeps the running sums of every step in
    # it: one 7-step call gives the same averages as 7 calls of one step, and the mean of their moments
    from paper_1810_07803_amd import hrlb

    say(f"[average] small-case path, nx32 q4x4 precision={precision}")
    cases = []
    for _ in range(2):
        c, _ = make_pair(4, 4, 32, delta=1.0, uw=0.2, stretch_A=0.9, precision=precision, rounding=precision,
                         path=hrlb.HRLB_PATH_SMALL)
        assert c.kernel_path() == hrlb.HRLB_PATH_SMALL
        c.step(5)
        c.average_start()
        cases.append(c)
    acc = np.zeros((10, 32))
    for _ in range(7):
        cases[0].step(1)
        acc += cases[0].moments()[0]
    cases[1].step(7)
    fa, _, na = cases[0].average_read()
    fb, _, nb = cases[1].average_read()
    assert na == nb == 7
    assert cases[0].steps_done() == cases[1].steps_done() == 12
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_allclose(fa, acc / 7, rtol=1e-14, atol=1e-15)

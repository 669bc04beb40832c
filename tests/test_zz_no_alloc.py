"""The allocation-free case (hrlb_init_case_static: the caller's memory holds the populations only,
the rest of the case lives in the library's static scratch) against the workspace case
(hrlb_init_case) with the same parameters: same kernels and plan, so the same bits, on two cases in a
row (the second smaller), in FP64 and in FP32 storage."""
import numpy as np
import pytest

from hrlb_inputs import perturb
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _start(hrlb, q, kw, static):
    c = hrlb.Case(q, hrlb.make_params(**kw), static=static)
    return c


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_static_case_equals_the_workspace_case_on_two_calls_in_a_row(precision, rounding):
    from paper_1810_07803_amd import hrlb

    prev = None
    for Qx, Qy, nx, steps in ((8, 8, 128, 30), (4, 4, 64, 20)):
        say(f"[no-alloc] Q{Qx}x{Qy} nx={nx} precision={precision}: static case vs workspace case")
        q = hrlb.Quadrature(Qx, Qy)
        kw = dict(delta=0.7, uw=0.3, ncell=nx, stretch_A=0.9, precision=precision, rounding=rounding, seed=17)
        ref = _start(hrlb, q, kw, False)
        sta = _start(hrlb, q, kw, True)
        if prev is not None:
            # the earlier static case was replaced: its calls fail cleanly
            with pytest.raises(hrlb.HrlbError) as ei:
                prev.step(1)
            assert ei.value.status == hrlb.HRLB_E_INVALID
        s0 = ref.get_state()
        s0 = np.stack([perturb(s0[0], 0.05, 5), perturb(s0[1], 0.05, 6)])
        ref.set_state(s0)
        sta.set_state(s0)
        ref.step(steps)
        sta.step(steps)
        st_r, inf_r = ref.run_to_steady(1e-300, 200, 100)
        st_s, inf_s = sta.run_to_steady(1e-300, 200, 100)
        np.testing.assert_array_equal(ref.get_state(), sta.get_state())
        fr, xr, pr, wr = ref.moments()
        fs, xs, ps, ws = sta.moments()
        np.testing.assert_array_equal(fr, fs)
        np.testing.assert_array_equal(wr, ws)
        assert pr == ps and st_r == st_s
        assert inf_r.residual == inf_s.residual and inf_r.pxy_drift == inf_s.pxy_drift
        say(f"   equal bit for bit after {steps + 200} steps (residual {inf_s.residual:.3e}, Pi {ps:.9f})")
        prev = sta


def test_static_case_beyond_the_scratch_is_rejected():
    from paper_1810_07803_amd import hrlb

    say("[no-alloc] nx=65536 Q16x8: auxiliary data beyond the 32 MiB scratch")
    q = hrlb.Quadrature(16, 8)
    with pytest.raises(hrlb.HrlbError) as ei:
        hrlb.Case(q, hrlb.make_params(delta=1.0, uw=0.1, ncell=65536, precision=1), static=True)
    assert ei.value.status == hrlb.HRLB_E_INVALID
    assert "scratch" in str(ei.value)

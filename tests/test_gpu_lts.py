"""Local time steps (steady-state acceleration, not in the paper) on the GPU: parity with the oracle
over checked steps (so the mass rescaling runs), the same steady state as the global time step in
fewer steps, batches that mix local-step and global-step cases, and a served local-step solve."""
import numpy as np
import pytest

from hrlb_inputs import perturb
from tests.gpu_helpers import moment_errs, parity, say

pytestmark = pytest.mark.gpu


def _lts_pair(Qx, Qy, nx, *, precision=0, rounding=0, cap=64.0, **kw):
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    orc = OracleProblem(Qx, Qy, nx, local_dt_cap=cap, **kw)
    q = hrlb.Quadrature(Qx, Qy, orc.Nx, orc.Ny)
    case = hrlb.Case(q, hrlb.make_params(delta=kw["delta"], uw=kw["uw"], ncell=nx, stretch_A=kw.get("stretch_A", 0.0),
                                         omega=kw.get("omega", 0.7), precision=precision, rounding=rounding,
                                         dt=orc.dt, seed=91, half_channel=int(kw.get("half_channel", False)),
                                         local_dt_cap=cap))
    case._quad_ref = q
    return case, orc


@pytest.mark.parametrize("precision,rounding,tol", [(0, 0, 1e-12), (1, 1, 1e-5)])
def test_local_time_steps_match_the_oracle_over_checked_steps(precision, rounding, tol):
    say(f"[lts] Q8x7 nx=132 half, A=0.98, 40 steps checked every 10, precision={precision}")
    kw = dict(delta=0.5, uw=0.4, omega=0.8, stretch_A=0.98, half_channel=True)
    case, orc = _lts_pair(8, 7, 132, precision=precision, rounding=rounding, **kw)
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.05, 51), perturb(chi, 0.05, 52)
    case.set_state(np.stack([phi, chi]))
    st, info = case.run_to_steady(1e-300, 40, 10)
    _, res = orc.step(phi, chi, 40, 10, 0.0)
    say(f"   steps {info.steps} residual {info.residual:.6e} vs {res:.6e}")
    assert info.steps == 40
    assert parity(case.get_state(), phi, chi, case.moments()[0], orc.moments(phi, chi), tol)
    assert info.residual == pytest.approx(res, rel=max(tol, 1e-10))
    assert orc.mass(phi) == pytest.approx(float(np.sum(orc.J * orc.deta)), rel=1e-14)


def test_local_time_steps_reach_the_global_steady_state_faster():
    from paper_1810_07803_amd import hrlb

    kw = dict(delta=1.0, uw=2 ** 0.5, ncell=16, stretch_A=0.98, omega=0.66, half_channel=1)
    q = hrlb.Quadrature(7, 7, 6, 6)
    g = hrlb.Case(q, hrlb.make_params(**kw))
    loc = hrlb.Case(q, hrlb.make_params(local_dt_cap=64.0, **kw))
    sg, ig = g.run_to_steady(1e-9, 400000, 500)
    sl, il = loc.run_to_steady(1e-9, 400000, 500)
    fg, _, pig, _ = g.moments()
    fl, _, pil, _ = loc.moments()
    say(f"[lts] HHLB(6;7) S=16 A=0.98 delta=1: global {ig.steps} steps, local {il.steps} steps; "
        f"Pi {pig:.12f} vs {pil:.12f}")
    assert sg == 0 and sl == 0
    assert il.steps * 4 < ig.steps
    assert moment_errs(fl, fg, 1e-8)
    assert pil == pytest.approx(pig, rel=1e-8)


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_batch_mixing_local_and_global_steps_is_bitwise_alone(precision, rounding):
    # checked steps re-analyse every instance of a launch that holds a local-step case: the global-step
    # instances must come out bit for bit as in a batch of their own
    from paper_1810_07803_amd import hrlb

    shapes = [(4, 4, 64, 64.0), (8, 7, 132, 0.0), (8, 7, 100, 16.0), (4, 8, 36, 0.0)]
    say(f"[lts] batch of local-step and global-step cases, precision={precision}")

    def cases():
        out = []
        for k, (Qx, Qy, nx, cap) in enumerate(shapes):
            q = hrlb.Quadrature(Qx, Qy)
            c = hrlb.Case(q, hrlb.make_params(delta=0.3, uw=0.4, ncell=nx, stretch_A=0.95, precision=precision,
                                              rounding=rounding, seed=70 + k, local_dt_cap=cap))
            c._quad_ref = q
            out.append(c)
        return out

    alone = cases()
    for c in alone:
        b1 = hrlb.Batch([c])
        for _ in range(3):
            b1.step(10, check=True)
    mixed = cases()
    b = hrlb.Batch(mixed)
    for _ in range(3):
        b.step(10, check=True)
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a.get_state(), m.get_state())
        np.testing.assert_array_equal(a.moments()[0], m.moments()[0])


def test_served_local_step_solve_equals_alone():
    from paper_1810_07803_amd import hrlb

    kw = dict(delta=1.0, uw=0.5, ncell=48, stretch_A=0.98, half_channel=1, local_dt_cap=64.0)
    q = hrlb.Quadrature(4, 4)
    alone = hrlb.Case(q, hrlb.make_params(**kw))
    st, info = alone.run_to_steady(1e-4, 20000, 100, hrlb.HRLB_STOP_PXY)
    srv = hrlb.Server(64 << 20, max_active=4, check_every=100, max_bypass=2, precision=0)
    rid = srv.submit(4, 4, hrlb.make_params(**kw), tol=1e-4, max_steps=20000)
    # a global-step solve resident at the same time
    srv.submit(8, 4, hrlb.make_params(delta=0.5, uw=0.2, ncell=64, stretch_A=0.9), tol=1e-4, max_steps=20000)
    while srv.pump().active:
        pass
    info_s, f_served, _ = srv.request(rid)
    say(f"[lts] served steps {info_s.steps} alone {info.steps}")
    assert info_s.state == hrlb.HRLB_REQ_DONE and info_s.steps == info.steps
    np.testing.assert_array_equal(f_served, alone.moments()[0])

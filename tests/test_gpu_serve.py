"""Serving loop with continuous batching: solves submitted while others are resident are admitted as
slots and arena memory free up, their steps share launches, and every result is the same, bit for
bit, as the same solve run alone with hrlb_run_to_steady.  One solve is also checked against the
oracle run to the same stop."""
import numpy as np
import pytest

from tests.gpu_helpers import moment_errs, say

pytestmark = pytest.mark.gpu

# (Qx, Qy, Nx, delta, u_w, omega, A): different velocity sets, grids and physics
REQS = [
    (4, 4, 32, 1.0, 0.05, 0.7, 0.0),
    (8, 4, 64, 0.3, 0.2, 0.5, 0.9),
    (4, 8, 48, 3.0, 0.1, 1.0, 0.5),
    (8, 8, 40, 0.05, 0.4, 0.8, 0.9),
    (4, 4, 64, 10.0, 0.3, 0.66, 0.9),
    (16, 4, 32, 0.5, 0.15, 0.75, 0.0),
]
CHECK_EVERY = 100
MAX_STEPS = 6000
TOL = 2e-3  # P_xy drift rate (per unit time): reached after a few hundred to a few thousand steps


def _params(k, precision, rounding):
    from paper_1810_07803_amd import hrlb

    Qx, Qy, nx, delta, uw, omega, A = REQS[k]
    return hrlb.make_params(delta=delta, uw=uw, ncell=nx, stretch_A=A, omega=omega, precision=precision,
                            rounding=rounding, seed=1000 + k)


def _alone(k, precision, rounding):
    from paper_1810_07803_amd import hrlb

    Qx, Qy = REQS[k][:2]
    q = hrlb.Quadrature(Qx, Qy)
    c = hrlb.Case(q, _params(k, precision, rounding))
    st, info = c.run_to_steady(TOL, MAX_STEPS, CHECK_EVERY, hrlb.HRLB_STOP_PXY)
    f, x, pi, _ = c.moments()
    return st, info, f, x, pi


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_served_results_equal_alone_bitwise(precision, rounding):
    from paper_1810_07803_amd import hrlb

    say(f"[serve] {len(REQS)} requests, precision={precision}, check_every={CHECK_EVERY}, tol={TOL}")
    sizes = [hrlb.workspace_bytes(hrlb.Quadrature(r[0], r[1]), _params(k, precision, rounding))
             for k, r in enumerate(REQS)]
    # room for about three solves at once: later arrivals wait for memory
    arena = int(sum(sorted(sizes)[-3:]) * 1.2) + (256 << 10)
    srv = hrlb.Server(arena, max_active=4, check_every=CHECK_EVERY, max_bypass=2, precision=precision)
    ids = []
    for k in range(3):
        Qx, Qy = REQS[k][:2]
        ids.append(srv.submit(Qx, Qy, _params(k, precision, rounding), tol=TOL, max_steps=MAX_STEPS))
    max_resident, rounds = 0, 0
    for _ in range(3):
        st = srv.pump()
        max_resident = max(max_resident, st.active)
        rounds += 1
    for k in range(3, len(REQS)):  # arrive while the first ones are resident
        Qx, Qy = REQS[k][:2]
        ids.append(srv.submit(Qx, Qy, _params(k, precision, rounding), tol=TOL, max_steps=MAX_STEPS))
    while True:
        st = srv.pump()
        rounds += 1
        max_resident = max(max_resident, st.active)
        assert st.arena_used <= arena
        if st.waiting == 0 and st.active == 0:
            break
        assert rounds < 10 * MAX_STEPS // CHECK_EVERY
    say(f"   rounds {rounds}, most resident at once {max_resident}, done {st.done}, failed {st.failed}")
    assert st.done == len(REQS) and st.failed == 0
    assert max_resident >= 2
    overlapped = 0
    infos = []
    for k, rid in enumerate(ids):
        info, f, x = srv.request(rid)
        infos.append(info)
        st_a, info_a, f_a, x_a, pi_a = _alone(k, precision, rounding)
        say(f"   req {k}: status {info.status} steps {info.steps} (alone {info_a.steps}), Pi {info.Pi:.12f}, "
            f"waited {info.t_admit - info.t_arrival:.3f}s, served {info.t_done - info.t_admit:.3f}s")
        assert info.status == st_a
        assert info.steps == info_a.steps
        np.testing.assert_array_equal(f, f_a)
        np.testing.assert_array_equal(x, x_a)
        assert info.Pi == pi_a
        assert info.t_arrival <= info.t_admit <= info.t_done
    for a in range(len(infos)):
        for b in range(a + 1, len(infos)):
            if infos[a].t_admit < infos[b].t_done and infos[b].t_admit < infos[a].t_done:
                overlapped += 1
    assert overlapped >= 1
    # released requests are forgotten
    srv.request(ids[0], release=True)
    with pytest.raises(hrlb.HrlbError):
        srv.request(ids[0])
    srv.free()


def test_served_solve_matches_oracle_at_the_same_stop():
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    say("[serve] request 0 vs the oracle run for the same number of steps (fp64)")
    Qx, Qy, nx, delta, uw, omega, A = REQS[0]
    srv = hrlb.Server(64 << 20, max_active=2, check_every=CHECK_EVERY, precision=0)
    rid = srv.submit(Qx, Qy, _params(0, 0, 0), tol=TOL, max_steps=MAX_STEPS)
    while True:
        st = srv.pump()
        if st.active == 0 and st.waiting == 0:
            break
    info, f, _ = srv.request(rid)
    orc = OracleProblem(Qx, Qy, nx, stretch_A=A, delta=delta, uw=uw, omega=omega)
    phi, chi = orc.init_state()
    orc.step(phi, chi, info.steps)
    say(f"   steps {info.steps}")
    assert moment_errs(f, orc.moments(phi, chi), 1e-12)
    srv.free()


def test_served_with_the_pxy_error_rule_equals_alone():
    # the serving configuration of the benchmark: FP32 with stochastic rounding, local time steps (cap
    # 64), CFL 1, the P_xy error rule checked every 250 steps; every request stops at the same step, with
    # the same estimate and the same fields, as the same solve alone
    from paper_1810_07803_amd import hrlb

    say("[serve] P_xy error rule, FP32, local steps, CFL 1: served vs alone")
    every, tol, cap = 250, 3e-6, 20000

    def params(k):
        Qx, Qy, nx, delta, uw, omega, A = REQS[k]
        return hrlb.make_params(delta=delta, uw=uw, ncell=nx, stretch_A=A, omega=omega, precision=1,
                                rounding=1, seed=2000 + k, local_dt_cap=64.0, cfl=1.0)

    srv = hrlb.Server(256 << 20, max_active=8, check_every=every, max_bypass=2, precision=1)
    ids = [srv.submit(REQS[k][0], REQS[k][1], params(k), tol=tol, max_steps=cap, stop_rule=hrlb.HRLB_STOP_PXY_ERR)
           for k in range(len(REQS))]
    while True:
        st = srv.pump()
        if st.waiting == 0 and st.active == 0:
            break
    for k, rid in enumerate(ids):
        info, f, _ = srv.request(rid)
        c = hrlb.Case(hrlb.Quadrature(REQS[k][0], REQS[k][1]), params(k))
        st_a, info_a = c.run_to_steady(tol, cap, every, hrlb.HRLB_STOP_PXY_ERR)
        say(f"   req {k}: status {info.status} steps {info.steps} (alone {info_a.steps}), "
            f"estimate {info.pxy_err:.2e} (alone {info_a.pxy_err:.2e})")
        assert info.status == st_a and info.steps == info_a.steps
        assert info.pxy_err == info_a.pxy_err
        np.testing.assert_array_equal(f, c.moments()[0])
    srv.free()

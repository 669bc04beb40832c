"""The small-case path (one workgroup holds a whole case in LDS and runs many steps per launch):
element-by-element parity with the oracle in every combination of the method it serves (full and half
channel, collisionless, tabulated law, hot wall, local time steps with checked steps, FP64 and FP32),
agreement with the tiled path, the same bits alone and in batches that mix both paths, the plain FP64
case run to its steady state, graph replays, and the errors of a case that does not fit."""
import math

import numpy as np
import pytest

from hrlb_inputs import perturb
from tests.gpu_helpers import moment_errs, parity, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def _case(hrlb, Qx, Qy, nx, path, orc=None, **kw):
    q = hrlb.Quadrature(Qx, Qy, None if orc is None else orc.Nx, None if orc is None else orc.Ny)
    c = hrlb.Case(q, hrlb.make_params(ncell=nx, kernel_path=path, **kw))
    c._quad_ref = q
    return c


def _oracle_pair(Qx, Qy, nx, *, precision=0, rounding=0, path=2, table=None, lts=0.0, **kw):
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    okw = {k: v for k, v in kw.items() if k in ("stretch_A", "delta", "uw", "Tw", "omega")}
    orc = OracleProblem(Qx, Qy, nx, half_channel=kw.get("half_channel", 0) == 1, visc_table=table,
                        local_dt_cap=lts, **okw)
    c = _case(hrlb, Qx, Qy, nx, path, orc, precision=precision, rounding=rounding, dt=orc.dt, seed=13,
              visc_table=table, local_dt_cap=lts, **kw)
    return c, orc


CASES = [  # name, Qx, Qy, nx, steps, kw
    ("couette_nx32_q4x4", 4, 4, 32, 50, dict(delta=1.0, uw=0.05, omega=0.7)),
    ("stretched_nx24_q4x3", 4, 3, 24, 40, dict(delta=0.3, uw=0.4, omega=0.8, stretch_A=0.9)),
    ("half_nx16_q4x4_A098", 4, 4, 16, 60, dict(delta=1.0, uw=2 ** 0.5, omega=0.66, stretch_A=0.98, half_channel=1)),
    ("collisionless_nx16_q4x3", 4, 3, 16, 40, dict(delta=0.0, uw=0.4)),
    ("hot_wall_nx20_q4x4", 4, 4, 20, 40, dict(delta=1.0, uw=1.2, Tw=2.0, stretch_A=0.9)),
    ("smallest_nx8_q3x3", 3, 3, 8, 30, dict(delta=1.0, uw=0.4, stretch_A=0.9)),
]


@pytest.mark.parametrize("precision,rounding,tol", [(0, 0, FP64_TOL), (1, 1, FP32_TOL), (1, 0, FP32_TOL)])
@pytest.mark.parametrize("name,Qx,Qy,nx,steps,kw", CASES)
def test_small_path_fixed_step_parity(name, Qx, Qy, nx, steps, kw, precision, rounding, tol):
    say(f"[small] {name} precision={precision}: {steps} steps in launches of 1, 7 and the rest")
    c, orc = _oracle_pair(Qx, Qy, nx, precision=precision, rounding=rounding, **kw)
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.05, 91), perturb(chi, 0.05, 92)
    c.set_state(np.stack([phi, chi]))
    c.step(1)
    c.step(7)
    c.step(steps - 8)
    orc.step(phi, chi, steps)
    f_orc = orc.moments(phi, chi)
    f_gpu, _, pi, shear = c.moments()
    assert parity(c.get_state(), phi, chi, f_gpu, f_orc, tol)
    assert c.steps_done() == steps
    if orc.uw != 0:
        assert pi == pytest.approx(orc.Pi(f_orc), rel=max(tol, 1e-12))
    _, _, info = orc.rhs(phi, chi)
    assert shear[1] == pytest.approx(info[3], rel=max(tol, 1e-11), abs=1e-15)


@pytest.mark.parametrize("precision,rounding,tol", [(0, 0, FP64_TOL), (1, 1, FP32_TOL)])
def test_small_path_tabulated_law(precision, rounding, tol):
    rng = np.random.default_rng(3)
    T = np.array([0.5, 0.8, 0.95, 1.02, 1.1, 1.4, 2.0])
    mu = 1.3 * T ** 0.7 * (1 + rng.uniform(-0.05, 0.05, len(T)))
    table = list(zip(T, mu, 2.0 / 3.0 * (1 + rng.uniform(-0.05, 0.05, len(T)))))
    say(f"[small] tabulated law, precision={precision}")
    c, orc = _oracle_pair(4, 4, 32, precision=precision, rounding=rounding, table=table, delta=0.7, uw=0.45,
                          stretch_A=0.9)
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.08, 93), perturb(chi, 0.08, 94)
    c.set_state(np.stack([phi, chi]))
    c.step(30)
    orc.step(phi, chi, 30)
    assert parity(c.get_state(), phi, chi, c.moments()[0], orc.moments(phi, chi), tol)


@pytest.mark.parametrize("precision,rounding,tol", [(0, 0, FP64_TOL), (1, 1, FP32_TOL)])
def test_small_path_local_time_steps_over_checked_steps(precision, rounding, tol):
    say(f"[small] local time steps, half channel A = 0.98, checks every 10 steps, precision={precision}")
    c, orc = _oracle_pair(4, 4, 24, precision=precision, rounding=rounding, lts=64.0, delta=0.5, uw=0.4,
                          omega=0.8, stretch_A=0.98, half_channel=1)
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.05, 95), perturb(chi, 0.05, 96)
    c.set_state(np.stack([phi, chi]))
    st, info = c.run_to_steady(1e-300, 40, 10)
    _, res = orc.step(phi, chi, 40, 10, 0.0)
    say(f"   residual {info.residual:.6e} vs {res:.6e}")
    assert info.steps == 40
    assert parity(c.get_state(), phi, chi, c.moments()[0], orc.moments(phi, chi), tol)
    assert info.residual == pytest.approx(res, rel=max(tol, 1e-10))


@pytest.mark.parametrize("rounding,half", [(1, 0), (0, 0), (1, 1)])
def test_small_path_several_items_per_thread(rounding, half):
    # FP32, Q4x3, 64 cells: four lanes per cell in the analysis and 24 x 16 = 384 update items for 256
    # threads, so half of the threads update two (velocity, strip) items and their wall partials add up
    # over both; checked steps (residual, mass) every 10 steps
    from paper_1810_07803_amd import hrlb

    say(f"[small] FP32 Q4x3 nx64 (two update items per thread), rounding={rounding}, half={half}")
    c, orc = _oracle_pair(4, 3, 64, precision=1, rounding=rounding, delta=0.4, uw=0.35, omega=0.75,
                          stretch_A=0.9, half_channel=half)
    assert c.kernel_path() == hrlb.HRLB_PATH_SMALL
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.05, 97), perturb(chi, 0.05, 98)
    c.set_state(np.stack([phi, chi]))
    st, info = c.run_to_steady(1e-300, 30, 10)
    _, res = orc.step(phi, chi, 30, 10, 0.0)
    say(f"   residual {info.residual:.6e} vs {res:.6e}")
    assert info.steps == 30
    f_orc = orc.moments(phi, chi)
    f_gpu, _, pi, shear = c.moments()
    assert parity(c.get_state(), phi, chi, f_gpu, f_orc, FP32_TOL)
    assert pi == pytest.approx(orc.Pi(f_orc), rel=FP32_TOL)
    # measured: within 7e-7 of the oracle's residual
    assert info.residual == pytest.approx(res, rel=FP32_TOL)


@pytest.mark.parametrize("precision,rounding,nx,tol", [(0, 0, 64, FP64_TOL), (1, 1, 128, FP32_TOL)])
def test_small_path_beyond_64_kib_of_lds(precision, rounding, nx, tol):
    # Q4x4 with 64 cells in FP64 or 128 in FP32 needs about 125 KB of LDS: the automatic choice takes
    # the small path as long as the device gives a workgroup that much (160 KB on MI355X)
    import time

    import torch

    from paper_1810_07803_amd import hrlb

    say(f"[small] Q4x4 nx{nx} precision={precision}: more than 64 KB of LDS")
    c, orc = _oracle_pair(4, 4, nx, precision=precision, rounding=rounding, path=hrlb.HRLB_PATH_AUTO, delta=0.5,
                          uw=0.3, omega=0.7, stretch_A=0.9)
    assert c.kernel_path() == hrlb.HRLB_PATH_SMALL
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.05, 99), perturb(chi, 0.05, 100)
    c.set_state(np.stack([phi, chi]))
    c.step(20)
    orc.step(phi, chi, 20)
    assert parity(c.get_state(), phi, chi, c.moments()[0], orc.moments(phi, chi), tol)
    # time per step against the tiled path (reported, not asserted)
    t = {}
    for path in (hrlb.HRLB_PATH_SMALL, hrlb.HRLB_PATH_TILED):
        k = _case(hrlb, 4, 4, nx, path, precision=precision, rounding=rounding, delta=0.5, uw=0.3, stretch_A=0.9)
        k.step(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k.step(1000)
        torch.cuda.synchronize()
        t[path] = (time.perf_counter() - t0) / 1000 * 1e6
    say(f"   us per step: small {t[hrlb.HRLB_PATH_SMALL]:.1f}, tiled {t[hrlb.HRLB_PATH_TILED]:.1f}")


def test_small_and_tiled_paths_agree():
    from paper_1810_07803_amd import hrlb

    say("[small] small vs tiled path, FP64, Q4x4 nx32, 200 steps")
    kw = dict(delta=1.0, uw=0.3, stretch_A=0.9, omega=0.7)
    a = _case(hrlb, 4, 4, 32, hrlb.HRLB_PATH_SMALL, **kw)
    b = _case(hrlb, 4, 4, 32, hrlb.HRLB_PATH_TILED, **kw)
    a.step(200)
    b.step(200)
    sa, sb = a.get_state(), b.get_state()
    assert np.max(np.abs(sa - sb)) / np.max(np.abs(sb)) < 1e-13
    assert moment_errs(a.moments()[0], b.moments()[0], 1e-13)


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_batch_mixing_small_and_tiled_cases_is_bitwise_alone(precision, rounding):
    from paper_1810_07803_amd import hrlb

    shapes = [(4, 4, 32, 0), (8, 8, 96, 0), (3, 3, 8, 1), (4, 3, 16, 0)]
    say(f"[small] batch of small and tiled cases, precision={precision}")

    def cases():
        out = []
        for k, (Qx, Qy, nx, half) in enumerate(shapes):
            out.append(_case(hrlb, Qx, Qy, nx, hrlb.HRLB_PATH_AUTO, delta=0.4 + k, uw=0.2, stretch_A=0.9,
                             precision=precision, rounding=rounding, seed=40 + k, half_channel=half,
                             local_dt_cap=64.0 if k == 3 else 0.0))
        return out

    alone = cases()
    for c in alone:
        c.run_to_steady(1e-300, 30, 15)
    mixed = cases()
    b = hrlb.Batch(mixed)
    b.set_streams(2)
    b.step(15, check=True)
    b.step(15, check=True)
    res, pxy = b.poll()
    for k, (a, m) in enumerate(zip(alone, mixed)):
        np.testing.assert_array_equal(a.get_state(), m.get_state())
        np.testing.assert_array_equal(a.moments()[0], m.moments()[0])
        assert a.steps_done() == m.steps_done() == 30


def test_small_path_graph_replay_matches_direct_launches():
    from paper_1810_07803_amd import hrlb

    say("[small] graph replays of 10-step blocks vs direct launches")
    kw = dict(delta=1.0, uw=0.2, stretch_A=0.9, precision=1, rounding=1, seed=7, local_dt_cap=32.0)
    a = _case(hrlb, 4, 4, 32, hrlb.HRLB_PATH_SMALL, **kw)
    b = _case(hrlb, 4, 4, 32, hrlb.HRLB_PATH_SMALL, **kw)
    b.set_graph_steps(10)
    for _ in range(3):
        a.run_to_steady(1e-300, 20, 10)
        b.run_to_steady(1e-300, 20, 10)
        np.testing.assert_array_equal(a.get_state(), b.get_state())


def test_plain_fp64_case_to_steady_state_on_the_small_path():
    # the plain method's workload: Nx = 32, HHLB(3;4) x HLB(3;4), delta = 1, u_w = 0.05, omega = 0.7
    say("[small] couette_nx32_q4x4 fp64 to residual 2e-14 on the small path")
    c, orc = _oracle_pair(4, 4, 32, path=2, delta=1.0, uw=0.05, omega=0.7)
    st, info = c.run_to_steady(2e-14, 80000, 100)
    assert st == 0, info.residual
    phi, chi = orc.init_state()
    taken, res = orc.step(phi, chi, 80000, 100, 2e-14)
    f_gpu, _, pi, _ = c.moments()
    f_orc = orc.moments(phi, chi)
    say(f"   gpu steps {info.steps} ({info.wall_s:.3f} s) oracle steps {taken}; Pi {pi:.15f} vs {orc.Pi(f_orc):.15f}")
    assert moment_errs(f_gpu, f_orc, 1e-12)
    assert pi == pytest.approx(orc.Pi(f_orc), rel=1e-12)
    assert abs(info.mass_drift) < 1e-12


def test_cases_that_do_not_fit_are_refused_the_small_path():
    from paper_1810_07803_amd import hrlb

    q = hrlb.Quadrature(8, 8)
    with pytest.raises(hrlb.HrlbError) as ei:
        hrlb.Case(q, hrlb.make_params(delta=1.0, uw=0.1, ncell=256, kernel_path=hrlb.HRLB_PATH_SMALL))
    assert ei.value.status == hrlb.HRLB_E_INVALID
    with pytest.raises(hrlb.HrlbError):
        hrlb.Case(q, hrlb.make_params(delta=1.0, uw=0.1, ncell=32, kernel_path=7))

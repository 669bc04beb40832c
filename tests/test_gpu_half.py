"""The half-channel formulation (point symmetry of Sec. II at x = 0) on the GPU: element-by-element
parity with the oracle's half channel, agreement with the GPU full channel of twice the cells,
batches that mix half and full cases, and the steady state against the oracle."""
import numpy as np
import pytest

from hrlb_inputs import perturb
from tests.gpu_helpers import make_pair, moment_errs, parity, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5

CASES = [  # name, Qx, Qy, ncell, steps, kw
    ("half_nx16_q4x4_uniform", 4, 4, 16, 40, dict(delta=1.0, uw=0.05, omega=0.7)),
    ("half_nx132_q8x7_stretched", 8, 7, 132, 20, dict(delta=0.5, uw=0.3, omega=0.8, stretch_A=0.9)),
    ("half_nx68_q16x8_stretched", 16, 8, 68, 10, dict(delta=0.1, uw=0.2, omega=0.66, stretch_A=0.9)),
    ("half_collisionless_nx24_q4x3", 4, 3, 24, 30, dict(delta=0.0, uw=0.4)),
]


def _run(name, Qx, Qy, ncell, steps, tol, *, precision=0, rounding=0, **kw):
    say(f"[half] {name}: Qx={Qx} Qy={Qy} ncell={ncell} steps={steps} precision={precision} rounding={rounding} {kw}")
    case, orc = make_pair(Qx, Qy, ncell, precision=precision, rounding=rounding, half_channel=True, seed=21, **kw)
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.05, 31), perturb(chi, 0.05, 32)
    case.set_state(np.stack([phi, chi]))
    case.step(steps)
    orc.step(phi, chi, steps)
    st = case.get_state()
    f_gpu, x, pi_gpu, shear = case.moments()
    f_orc = orc.moments(phi, chi)
    ok = parity(st, phi, chi, f_gpu, f_orc, tol)
    np.testing.assert_allclose(x, orc.x, rtol=0, atol=1e-15)
    _, _, info = orc.rhs(phi, chi)
    return ok, (pi_gpu, orc.Pi(f_orc)), (shear, info)


@pytest.mark.parametrize("name,Qx,Qy,ncell,steps,kw", CASES)
def test_half_channel_fixed_step_parity_fp64(name, Qx, Qy, ncell, steps, kw):
    ok, (pi_g, pi_o), (shear, info) = _run(name, Qx, Qy, ncell, steps, FP64_TOL, **kw)
    assert ok
    assert pi_g == pytest.approx(pi_o, rel=1e-12, abs=1e-15)
    # the one wall, at x = 1/2 (reported in both slots)
    assert shear[1] == pytest.approx(info[3], rel=1e-11, abs=1e-15) and shear[0] == shear[1]


@pytest.mark.parametrize("rounding", [0, 1])
def test_half_channel_fixed_step_parity_fp32(rounding):
    name, Qx, Qy, ncell, steps, kw = CASES[2]
    ok, *_ = _run(name + "_fp32", Qx, Qy, ncell, steps, FP32_TOL, precision=1, rounding=rounding, **kw)
    assert ok


def test_half_channel_is_the_right_half_of_the_full_channel_on_gpu():
    # the same flow with half the cells: the GPU half channel against the GPU full channel of 2S cells
    S, steps = 100, 60
    say(f"[half] GPU half nx{S} vs GPU full nx{2 * S}, q8x4, {steps} steps")
    kw = dict(delta=0.5, uw=0.3, omega=0.8, stretch_A=0.9)
    h, _ = make_pair(8, 4, S, half_channel=True, **kw)
    f, _ = make_pair(8, 4, 2 * S, **kw)
    assert h.dt == f.dt
    h.step(steps)
    f.step(steps)
    sh, sf = h.get_state(), f.get_state()
    e = np.max(np.abs(sh - sf[:, :, S:])) / np.max(np.abs(sf))
    fh, xh, pih, shh = h.moments()
    ff, xf, pif, shf = f.moments()
    say(f"   state diff {e:.2e}; Pi {pih:.15f} vs {pif:.15f}")
    assert e < 1e-13
    np.testing.assert_allclose(xh, xf[S:], rtol=0, atol=1e-15)
    assert pih == pytest.approx(pif, rel=1e-12)
    assert shh[1] == pytest.approx(shf[1], rel=1e-12)


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_batch_mixing_half_and_full_cases_is_bitwise_alone(precision, rounding):
    from paper_1810_07803_amd import hrlb

    shapes = [(4, 4, 64, True), (8, 7, 132, False), (8, 7, 132, True), (4, 8, 36, True)]
    say(f"[half] batch of half and full cases, precision={precision}")

    def cases():
        return [make_pair(Qx, Qy, nx, delta=0.3, uw=0.2, stretch_A=0.9, precision=precision, rounding=rounding,
                          seed=50 + k, half_channel=half)[0]
                for k, (Qx, Qy, nx, half) in enumerate(shapes)]

    alone = cases()
    for c in alone:
        c.step(15)
    mixed = cases()
    b = hrlb.Batch(mixed)
    b.step(15)
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a.get_state(), m.get_state())
        np.testing.assert_array_equal(a.moments()[0], m.moments()[0])


def test_half_channel_steady_state_against_oracle():
    # both sides run to a residual of 2e-14, where the distance to the fixed point (about the residual
    # over the slowest decay rate) is below 1e-12
    say("[half] steady state nx16 q4x4 fp64 (the right half of couette_nx32_q4x4) to residual 2e-14")
    case, orc = make_pair(4, 4, 16, delta=1.0, uw=0.05, omega=0.7, half_channel=True)
    st, info = case.run_to_steady(2e-14, 80000, 100)
    assert st == 0, info.residual
    phi, chi = orc.init_state()
    taken, res = orc.step(phi, chi, 80000, 100, 2e-14)
    assert res < 2e-14
    f_gpu, _, pi_gpu, _ = case.moments()
    f_orc = orc.moments(phi, chi)
    say(f"   gpu steps {info.steps} oracle steps {taken}; Pi {pi_gpu:.15f} vs {orc.Pi(f_orc):.15f}; "
        f"mass drift {info.mass_drift:.2e}")
    assert moment_errs(f_gpu, f_orc, 1e-12)
    assert pi_gpu == pytest.approx(orc.Pi(f_orc), rel=1e-12)
    assert abs(info.mass_drift) < 1e-12


def test_served_half_channel_solve_equals_alone():
    from paper_1810_07803_amd import hrlb

    kw = dict(delta=1.0, uw=0.5, ncell=24, stretch_A=0.95, half_channel=1)
    q = hrlb.Quadrature(4, 4)
    alone = hrlb.Case(q, hrlb.make_params(**kw))
    st, info = alone.run_to_steady(1e-4, 20000, 100, hrlb.HRLB_STOP_PXY)
    srv = hrlb.Server(64 << 20, max_active=4, check_every=100, max_bypass=2, precision=0)
    rid = srv.submit(4, 4, hrlb.make_params(**kw), tol=1e-4, max_steps=20000)
    srv.submit(8, 4, hrlb.make_params(delta=0.5, uw=0.2, ncell=64, stretch_A=0.9), tol=1e-4, max_steps=20000)
    while srv.pump().active:
        pass
    info_s, f_served, x_served = srv.request(rid)
    say(f"[half] served steps {info_s.steps} alone {info.steps}, Pi {info_s.Pi:.12f}")
    assert info_s.state == hrlb.HRLB_REQ_DONE and info_s.steps == info.steps
    f, x, pi, _ = alone.moments()
    np.testing.assert_array_equal(f_served, f)
    np.testing.assert_array_equal(x_served, x)
    assert info_s.Pi == pi

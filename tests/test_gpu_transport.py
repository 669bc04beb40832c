"""The tabulated transport law of eqs. (mun) and (interp) on the GPU: element-by-element parity with
the oracle while cell temperatures cross several table intervals, a table sampled from a power law
against that power law, batches mixing tabulated and power-law cases, and a served solve whose table
the caller dropped after submitting it."""
import gc

import numpy as np
import pytest

from hrlb_inputs import perturb
from tests.gpu_helpers import parity, say

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def _table(seed):
    """Rows (T_k, mu_k, Pr_k) with several nodes inside the 0.9-1.1 band that the perturbed start
    visits (none within 1e-3 of T_w = 1), steep and flat intervals, Pr within a few percent of 2/3."""
    rng = np.random.default_rng(seed)
    T = np.array([0.5, 0.91, 0.955, 0.985, 1.012, 1.04, 1.075, 1.6])
    mu = T ** 0.7 * np.exp(rng.uniform(-0.04, 0.04, len(T)))
    Pr = 2.0 / 3.0 * (1 + rng.uniform(-0.05, 0.05, len(T)))
    return list(zip(T, mu, Pr))


def _pair(Qx, Qy, nx, steps, *, precision=0, rounding=0, table, **kw):
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    orc = OracleProblem(Qx, Qy, nx, visc_table=table, **kw)
    q = hrlb.Quadrature(Qx, Qy, orc.Nx, orc.Ny)
    case = hrlb.Case(q, hrlb.make_params(delta=kw["delta"], uw=kw["uw"], ncell=nx, stretch_A=kw.get("stretch_A", 0.0),
                                         precision=precision, rounding=rounding, dt=orc.dt, seed=77,
                                         visc_table=table))
    case._quad_ref = q
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.08, 41), perturb(chi, 0.08, 42)
    case.set_state(np.stack([phi, chi]))
    case.step(steps)
    orc.step(phi, chi, steps)
    f_orc = orc.moments(phi, chi)
    tol = FP64_TOL if precision == 0 else FP32_TOL
    ok = parity(case.get_state(), phi, chi, case.moments()[0], f_orc, tol)
    return ok, f_orc[3]


@pytest.mark.parametrize("Qx,Qy,nx,steps,kw,min_intervals", [
    (8, 7, 132, 20, dict(delta=0.5, uw=0.3, stretch_A=0.9), 3),
    (4, 4, 64, 40, dict(delta=2.0, uw=0.45), 2),
])
def test_tabulated_law_fixed_step_parity_fp64(Qx, Qy, nx, steps, kw, min_intervals):
    table = _table(3)
    say(f"[table] Q{Qx}x{Qy} nx={nx} {steps} steps {kw}, {len(table)} rows")
    ok, T = _pair(Qx, Qy, nx, steps, table=table, **kw)
    rows = np.array([r[0] for r in table])
    visited = np.unique(np.searchsorted(rows, T, side="right"))
    say(f"   T in [{T.min():.4f}, {T.max():.4f}], {len(visited)} intervals")
    assert len(visited) >= min_intervals
    assert ok


@pytest.mark.parametrize("rounding", [0, 1])
def test_tabulated_law_fixed_step_parity_fp32(rounding):
    say(f"[table] fp32 rounding={rounding}")
    ok, _ = _pair(8, 7, 132, 20, precision=1, rounding=rounding, table=_table(4), delta=0.5, uw=0.3, stretch_A=0.9)
    assert ok


def test_power_law_table_equals_the_power_law_on_gpu():
    # samples of mu = c T^omega with constant Pr: every interval's exponent is omega
    from paper_1810_07803_amd import hrlb

    omega, Pr = 0.66, 2.0 / 3.0
    table = [(T, 2.5 * T ** omega, Pr) for T in (0.4, 0.8, 0.97, 1.05, 1.3, 2.2)]
    q = hrlb.Quadrature(8, 4)
    base = dict(delta=0.4, uw=0.35, ncell=100, stretch_A=0.9, Pr=Pr)
    a = hrlb.Case(q, hrlb.make_params(omega=omega, **base))
    b = hrlb.Case(q, hrlb.make_params(visc_table=table, **base))
    a.step(200)
    b.step(200)
    sa, sb = a.get_state(), b.get_state()
    e = np.max(np.abs(sa - sb)) / np.max(np.abs(sa))
    say(f"[table] power-law table vs power law after 200 steps: {e:.2e}")
    assert e < 1e-13


@pytest.mark.parametrize("precision,rounding", [(0, 0), (1, 1)])
def test_batch_mixing_tabulated_and_power_law_cases_is_bitwise_alone(precision, rounding):
    from paper_1810_07803_amd import hrlb

    tables = [_table(5), None, _table(6), None]
    shapes = [(4, 4, 64), (8, 7, 132), (8, 7, 100), (4, 8, 36)]
    say(f"[table] batch of tabulated and power-law cases, precision={precision}")

    def cases():
        out = []
        for k, ((Qx, Qy, nx), tab) in enumerate(zip(shapes, tables)):
            q = hrlb.Quadrature(Qx, Qy)
            c = hrlb.Case(q, hrlb.make_params(delta=0.3, uw=0.4, ncell=nx, stretch_A=0.9, precision=precision,
                                              rounding=rounding, seed=60 + k, visc_table=tab))
            c._quad_ref = q
            out.append(c)
        return out

    alone = cases()
    for c in alone:
        c.step(15)
    mixed = cases()
    b = hrlb.Batch(mixed)
    b.step(15)
    for a, m in zip(alone, mixed):
        np.testing.assert_array_equal(a.get_state(), m.get_state())


def test_served_solve_keeps_its_own_copy_of_the_table():
    from paper_1810_07803_amd import hrlb

    table = _table(8)
    kw = dict(delta=1.0, uw=0.3, ncell=48, stretch_A=0.9)
    q = hrlb.Quadrature(4, 4)
    alone = hrlb.Case(q, hrlb.make_params(visc_table=table, **kw))
    st, info = alone.run_to_steady(2e-3, 6000, 100, hrlb.HRLB_STOP_PXY)
    f_alone = alone.moments()[0]
    srv = hrlb.Server(64 << 20, max_active=4, check_every=100, max_bypass=2, precision=0)
    params = hrlb.make_params(visc_table=table, **kw)
    rid = srv.submit(4, 4, params, tol=2e-3, max_steps=6000)
    # the caller overwrites its table arrays before the solve is admitted (a server that read them
    # later would see NaN rows, which hrlb_init_case rejects)
    for c in params._visc_keep:
        c[:] = np.nan
    del params
    gc.collect()
    while srv.pump().active or srv.request(rid)[0].state == hrlb.HRLB_REQ_WAITING:
        pass
    info_s, f_served, _ = srv.request(rid, release=True)
    say(f"[table] served steps {info_s.steps} alone steps {info.steps}")
    assert info_s.state == hrlb.HRLB_REQ_DONE and info_s.steps == info.steps
    np.testing.assert_array_equal(f_served, f_alone)

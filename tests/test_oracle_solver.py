"""Pins for the oracle's full time step (paper Secs. II-III): invariants, symmetry, the
free-molecular closed form, the Navier-Stokes limit and time-step independence."""
import math

import numpy as np
import pytest

from oracle.oracle import OracleProblem


def _mirror_index(p):
    # velocity (h, i, j) -> (1-h, i, Qy-1-j), i.e. (p_x, p_y) -> (-p_x, -p_y)
    Qx, Qy = p.Qx, p.Qy
    idx = np.empty(p.nv, dtype=int)
    for v in range(p.nv):
        hi, j = divmod(v, Qy)
        h, i = divmod(hi, Qx)
        idx[v] = ((1 - h) * Qx + i) * Qy + (Qy - 1 - j)
    return idx


@pytest.mark.parametrize("Tw,A", [(1.0, 0.0), (1.0, 0.9), (1.3, 0.9)])
def test_rest_state_is_preserved(Tw, A):
    # walls at rest with the gas in their own equilibrium: every term of the step vanishes
    p = OracleProblem(4, 4, 16, stretch_A=A, delta=1.0, uw=0.0, Tw=Tw)
    phi, chi = p.init_state()
    phi0, chi0 = phi.copy(), chi.copy()
    p.step(phi, chi, 20)
    assert np.max(np.abs(phi - phi0)) <= 1e-14 * np.max(phi0)
    assert np.max(np.abs(chi - chi0)) <= 1e-14 * np.max(chi0)
    _, _, info = p.rhs(phi, chi)
    assert info[0] == pytest.approx(1.0, abs=1e-14) and info[1] == pytest.approx(1.0, abs=1e-14)


def test_mass_is_conserved_to_round_off():
    # zero wall mass flux (diffuse_nw) plus a conservative collision keep sum_s J_s deta n_s
    p = OracleProblem(4, 4, 16, stretch_A=0.9, delta=1.0, uw=0.3)
    phi, chi = p.init_state()
    m0 = p.mass(phi)
    p.step(phi, chi, 300)
    assert abs(p.mass(phi) - m0) <= 2e-14 * m0
    dphi, _, _ = p.rhs(phi, chi)
    assert abs(float(np.sum(p.J * p.deta * dphi.sum(axis=0)))) < 1e-12


def test_point_symmetry_of_the_couette_problem():
    # Sec. II: phi(-x, -p_x, -p_y) = phi(x, p_x, p_y); hence n, T, P_xy even and u_y, q odd
    p = OracleProblem(4, 4, 16, stretch_A=0.9, delta=1.0, uw=0.2)
    phi, chi = p.init_state()
    p.step(phi, chi, 200)
    mi = _mirror_index(p)
    assert np.max(np.abs(phi[mi][:, ::-1] - phi)) <= 1e-13 * np.max(phi)
    assert np.max(np.abs(chi[mi][:, ::-1] - chi)) <= 1e-13 * np.max(chi)
    f = p.moments(phi, chi)
    for k, parity in zip(range(10), (+1, -1, -1, +1, +1, +1, +1, +1, -1, -1)):
        scale = max(np.max(np.abs(f[k])), 1e-3)
        assert np.max(np.abs(f[k][::-1] - parity * f[k])) <= 1e-12 * scale, k


@pytest.mark.parametrize("Qx,Qy,S,A", [(4, 4, 24, 0.9), (8, 7, 20, 0.0)])
def test_half_channel_is_the_right_half_of_the_full_channel(Qx, Qy, S, A):
    # Sec. II: the symmetry (x, p_x, p_y) -> (-x, -p_x, -p_y) lets the right half [0, 1/2] stand for
    # the channel.  The half grid of equation (stretch) is the right half of the full grid with 2S
    # cells, and the mirrored ghosts at x = 0 reproduce the full channel's left neighbours, so both
    # runs agree to round-off (a wrong mirror index, grid or face at x = 0 breaks this at O(1e-3)).
    kw = dict(stretch_A=A, delta=1.0, uw=0.3, omega=0.7)
    h = OracleProblem(Qx, Qy, S, half_channel=True, **kw)
    f = OracleProblem(Qx, Qy, 2 * S, **kw)
    assert h.dt == f.dt
    np.testing.assert_allclose(h.x, f.x[S:], rtol=0, atol=1e-15)
    np.testing.assert_allclose(h.J * h.deta, f.J[S:] * f.deta, rtol=1e-15)
    ph, ch = h.init_state()
    pf, cf = f.init_state()
    h.step(ph, ch, 150)
    f.step(pf, cf, 150)
    assert np.max(np.abs(ph - pf[:, S:])) <= 1e-13 * np.max(np.abs(pf))
    assert np.max(np.abs(ch - cf[:, S:])) <= 1e-13 * np.max(np.abs(cf))
    mh, mf = h.moments(ph, ch), f.moments(pf, cf)
    assert abs(h.Pi(mh) - f.Pi(mf)) <= 1e-13 * abs(f.Pi(mf))
    assert abs(h.mass(ph) - 0.5 * f.mass(pf)) <= 1e-14
    # the wall at x = 1/2 sees the same n_w and momentum flux
    _, _, ih = h.rhs(ph, ch)
    _, _, iff = f.rhs(pf, cf)
    assert abs(ih[1] - iff[1]) <= 1e-13 and abs(ih[3] - iff[3]) <= 1e-13 * abs(iff[3])


def test_half_channel_conserves_mass_and_keeps_the_rest_state():
    # no mass crosses x = 0 (the mirrored fluxes cancel) nor the diffuse wall (diffuse_nw)
    p = OracleProblem(4, 4, 16, stretch_A=0.9, delta=1.0, uw=0.3, half_channel=True)
    phi, chi = p.init_state()
    m0 = p.mass(phi)
    p.step(phi, chi, 300)
    assert abs(p.mass(phi) - m0) <= 1e-13 * m0
    r = OracleProblem(4, 4, 16, stretch_A=0.9, delta=1.0, uw=0.0, half_channel=True)
    phi, chi = r.init_state()
    phi0 = phi.copy()
    r.step(phi, chi, 20)
    assert np.max(np.abs(phi - phi0)) <= 1e-14 * np.max(phi0)


def test_local_time_steps_reach_the_same_steady_state_in_fewer_steps():
    # local steps change the transient only: the fixed point R(f) = 0 at the rest-state mass is the
    # one the global time step reaches (A = 0.98 gives cells 24x apart in size)
    kw = dict(stretch_A=0.98, delta=1.0, uw=0.5, omega=0.7, half_channel=True)
    g = OracleProblem(4, 4, 16, **kw)
    loc = OracleProblem(4, 4, 16, local_dt_cap=64.0, **kw)
    pg, cg = g.init_state()
    pl, cl = loc.init_state()
    ng, rg = g.step(pg, cg, 200000, 200, 1e-10)
    nl, rl = loc.step(pl, cl, 200000, 200, 1e-10)
    assert rg < 1e-10 and rl < 1e-10
    assert nl * 4 < ng
    fg, fl = g.moments(pg, cg), loc.moments(pl, cl)
    for k in range(10):
        assert np.max(np.abs(fg[k] - fl[k])) <= 1e-8 * max(1.0, np.max(np.abs(fg[k])))
    assert abs(loc.Pi(fl) - g.Pi(fg)) <= 1e-8 * abs(g.Pi(fg))
    # every check rescales to the rest-state mass sum_s J_s deta
    assert loc.mass(pl) == pytest.approx(float(np.sum(loc.J * loc.deta)), rel=1e-14)


def test_local_time_steps_on_a_uniform_grid_are_the_global_step():
    # with equal cells every local step equals dt: the run differs from the global one only by the
    # mass rescaling at checks, which is 1 to round-off (the global step conserves mass)
    kw = dict(stretch_A=0.0, delta=1.0, uw=0.3)
    g = OracleProblem(4, 4, 16, **kw)
    loc = OracleProblem(4, 4, 16, local_dt_cap=64.0, **kw)
    pg, cg = g.init_state()
    pl, cl = loc.init_state()
    g.step(pg, cg, 300, 100)
    loc.step(pl, cl, 300, 100)
    assert np.max(np.abs(pg - pl)) <= 1e-13 * np.max(pg)


def test_local_time_steps_rescale_mass_at_every_check():
    # without checks the stretched-grid transient drifts in mass; with a check it is restored
    kw = dict(stretch_A=0.98, delta=1.0, uw=0.5, half_channel=True, local_dt_cap=64.0)
    p = OracleProblem(4, 4, 16, **kw)
    m0 = float(np.sum(p.J * p.deta))
    phi, chi = p.init_state()
    p.step(phi, chi, 50)
    assert abs(p.mass(phi) / m0 - 1) > 1e-6
    p.step(phi, chi, 10, 10)
    assert p.mass(phi) == pytest.approx(m0, rel=1e-14)


def test_free_molecular_limit_gives_pi_equal_one_over_sqrt_pi():
    # delta -> 0: each half-range stream carries its wall's Maxwellian, so n = 1,
    # T = 1 + u_w^2/3, P_xy = -u_w sqrt(2/pi) and equation (Pi) gives 1/sqrt(pi)
    uw = 0.1
    p = OracleProblem(4, 4, 16, delta=0.0, uw=uw)
    phi, chi = p.init_state()
    steps, res = p.step(phi, chi, 20000, 500, 1e-12)
    assert res < 1e-12
    f = p.moments(phi, chi)
    assert p.Pi(f) == pytest.approx(1 / math.sqrt(math.pi), abs=1e-12)
    np.testing.assert_allclose(f[0], 1.0, atol=1e-11)
    np.testing.assert_allclose(f[3], 1 + uw * uw / 3, atol=1e-11)
    np.testing.assert_allclose(f[2], 0.0, atol=1e-11)


@pytest.mark.slow
def test_navier_stokes_limit_linear_profile_and_slip():
    # large delta: Pi ~ 1/(delta + 2 sigma_P) with a viscous-slip coefficient near 1 (S model,
    # diffuse walls) and a linear bulk velocity profile
    sig = []
    for delta in (20.0, 40.0):
        p = OracleProblem(4, 4, 16, delta=delta, uw=0.05)
        phi, chi = p.init_state()
        steps, res = p.step(phi, chi, 40000, 500, 1e-11)
        assert res < 1e-11
        f = p.moments(phi, chi)
        Pi = p.Pi(f)
        sig.append((1 / Pi - delta) / 2)
        bulk = np.abs(p.x) < 0.3
        coef = np.polyfit(p.x[bulk], f[2][bulk], 1)
        resid = f[2][bulk] - np.polyval(coef, p.x[bulk])
        assert np.max(np.abs(resid)) < 2e-3 * np.max(np.abs(f[2]))
        # bulk shear rate u' = u_w/(1 + 2 sigma/delta) (u_y = 2 u' x)
        assert coef[0] == pytest.approx(2 * 0.05 / (1 + 2 * sig[-1] / delta), rel=2e-2)
    assert all(0.95 < s < 1.08 for s in sig), sig


def test_steady_state_does_not_depend_on_time_step():
    # the steady state is the fixed point R(f) = 0, independent of dt
    out = []
    for cfl in (0.5, 0.25):
        p = OracleProblem(4, 4, 16, stretch_A=0.9, delta=1.0, uw=0.1, cfl=cfl)
        phi, chi = p.init_state()
        steps, res = p.step(phi, chi, 40000, 200, 1e-12)
        assert res < 1e-12
        out.append(p.moments(phi, chi))
        dphi, dchi, _ = p.rhs(phi, chi)
        assert np.max(np.abs(dphi)) < 1e-10 * np.max(np.abs(phi)) / p.dt
    np.testing.assert_allclose(out[0], out[1], rtol=0, atol=2e-11)


def test_one_step_near_a_fixed_point_is_the_ssp_rk3_polynomial():
    # At a fixed point f* (R(f*) = 0) every stage of the third-order TVD Runge-Kutta scheme sits at f*,
    # so the step map linearises to I + dt J + (dt J)^2/2 + (dt J)^3/6 with J = DR(f*) (Sec. III
    # names the scheme; Shu & Osher 1988).  The rest state with walls at rest is an exact fixed point;
    # J v is formed by central differences of the oracle's right-hand side, independently of its step.
    p = OracleProblem(3, 3, 8, stretch_A=0.5, delta=1.0, uw=0.0, omega=0.7)
    phi0, chi0 = p.init_state()
    f0 = np.concatenate([phi0.ravel(), chi0.ravel()])
    n = phi0.size

    def R(f):
        dp, dc, _ = p.rhs(f[:n].reshape(phi0.shape), f[n:].reshape(chi0.shape))
        return np.concatenate([dp.ravel(), dc.ravel()])

    def step(f):
        a, b = f[:n].reshape(phi0.shape).copy(), f[n:].reshape(chi0.shape).copy()
        p.step(a, b, 1)
        return np.concatenate([a.ravel(), b.ravel()])

    assert np.max(np.abs(R(f0))) < 1e-15
    rng = np.random.default_rng(3)
    d = f0 * rng.uniform(-1.0, 1.0, size=f0.shape)
    # small enough that WENO's nonlinear weights stay at their linear values (the smoothness
    # indicators scale with the square of the perturbation against eps = 1e-6), large enough for
    # round-off
    eps = 2e-7

    def Jv(v):
        s = eps / max(np.max(np.abs(v / f0)), 1e-300)
        return (R(f0 + s * v) - R(f0 - s * v)) / (2 * s)

    z1 = p.dt * Jv(d)
    z2 = p.dt * Jv(z1)
    z3 = p.dt * Jv(z2)
    lhs = (step(f0 + eps * d) - step(f0 - eps * d)) / (2 * eps)
    rk3 = d + z1 + z2 / 2 + z3 / 6
    scale = np.max(np.abs(d))
    assert np.max(np.abs(z2)) > 1e-3 * scale and np.max(np.abs(z3)) > 1e-4 * scale  # terms are visible
    assert np.max(np.abs(lhs - rk3)) < 1e-7 * scale
    # a second-order scheme or a mis-weighted third stage would be far off
    assert np.max(np.abs(lhs - (d + z1 + z2 / 2))) > 1e3 * np.max(np.abs(lhs - rk3))


def test_time_marched_steady_state_is_the_zero_of_the_operator():
    # Brute force on a tiny case: Newton's method on R(f) = 0 with a finite-difference Jacobian and
    # the total mass fixed (the steady state is unique only up to mass) reaches the same state as
    # time marching to a residual of 1e-13.
    p = OracleProblem(4, 4, 8, stretch_A=0.5, delta=1.0, uw=0.2, omega=0.7)
    phi, chi = p.init_state()
    n = phi.size
    m0 = p.mass(phi)
    taken, res = p.step(phi, chi, 200000, 100, 1e-13)
    assert res < 1e-13, (taken, res)
    f_march = np.concatenate([phi.ravel(), chi.ravel()])

    def R(f):
        dp, dc, _ = p.rhs(f[:n].reshape(phi.shape), f[n:].reshape(chi.shape))
        return np.concatenate([dp.ravel(), dc.ravel()])

    wmass = np.zeros(2 * n)
    wmass[:n] = np.tile(p.J * p.deta, p.nv)  # mass = sum_s J_s deta sum_v phi_v,s
    a, b = p.init_state()
    f = np.concatenate([a.ravel(), b.ravel()])
    for _ in range(12):
        r = R(f)
        h = 1e-7 * max(np.max(np.abs(f)), 1e-12)
        Jm = np.empty((2 * n, 2 * n))
        for k in range(2 * n):
            e = np.zeros(2 * n)
            e[k] = h
            Jm[:, k] = (R(f + e) - R(f - e)) / (2 * h)
        # least squares on the operator plus the mass constraint
        A = np.vstack([Jm, wmass[None, :]])
        rhs = -np.concatenate([r, [wmass @ f - m0]])
        delta_f = np.linalg.lstsq(A, rhs, rcond=None)[0]
        f = f + delta_f
        if np.max(np.abs(delta_f)) < 1e-14 * np.max(np.abs(f)):
            break
    assert np.max(np.abs(R(f))) < 1e-11 * np.max(np.abs(f))
    assert np.max(np.abs(f - f_march)) < 1e-9 * np.max(np.abs(f_march))

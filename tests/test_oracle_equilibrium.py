"""Pins for the oracle's equilibrium truncations, moments, relaxation time and collision term
(paper Secs. II-III), checked against brute-force integrals and closed forms."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import quadrature as quad
from oracle.oracle import OracleProblem


def _half_moment(s, u, T, sign):
    """int over one half line of g(p,u,T) (sign*p)^s, by mp.quad (brute force)."""
    with mp.workdps(30):
        g = lambda p: mp.exp(-(p - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)
        if sign > 0:
            return float(mp.quad(lambda p: g(p) * p ** s, [0, 1, 4, mp.inf]))
        return float(mp.quad(lambda p: g(p) * (-p) ** s, [-mp.inf, -4, -1, 0]))


def _full_moment(l, u, T):
    with mp.workdps(30):
        g = lambda p: mp.exp(-(p - u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)
        return float(mp.quad(lambda p: g(p) * p ** l, [-mp.inf, u - 4, u, u + 4, mp.inf]))


@pytest.mark.parametrize("Qx,Nx,u,T", [(4, 3, 0.05, 1.02), (7, 6, -0.3, 0.8), (8, 7, 0.2, 1.3),
                                       (16, 10, 0.01, 1.05), (32, 10, 0.4, 1.1)])
def test_gx_recovers_half_range_moments(Qx, Nx, u, T):
    # Sec. III: sum_{i<=Q} g_{x,i} p_i^s equals int_0^inf g p^s dp for s <= N_x (each half)
    p = OracleProblem(Qx, 4, 8, Nx=Nx)
    g = p.gx(u, T)
    z = p.zx
    for s in range(Nx + 1):
        plus = float(np.sum(g[:Qx] * z ** s))
        minus = float(np.sum(g[Qx:] * z ** s))
        assert plus == pytest.approx(_half_moment(s, u, T, +1), rel=1e-13, abs=1e-15)
        assert minus == pytest.approx(_half_moment(s, u, T, -1), rel=1e-13, abs=1e-15)


def test_gx_equals_unique_vandermonde_solution_when_N_is_Q_minus_1():
    # with N = Q-1, the Q values on a half line are fixed by the Q moment conditions alone
    Q, u, T = 5, 0.17, 1.12
    p = OracleProblem(Q, 4, 8, Nx=Q - 1)
    g = p.gx(u, T)
    r = quad.half_range_rule(Q)
    with mp.workdps(60):
        V = mp.matrix([[z ** s for z in r.nodes] for s in range(Q)])
        for sign, sl in ((+1, slice(0, Q)), (-1, slice(Q, 2 * Q))):
            gg = lambda t: mp.exp(-(t - sign * u) ** 2 / (2 * T)) / mp.sqrt(2 * mp.pi * T)
            rhs = mp.matrix([mp.quad(lambda t: gg(t) * t ** s, [0, 1, 4, mp.inf]) for s in range(Q)])
            sol = mp.lu_solve(V, rhs)
            np.testing.assert_allclose(g[sl], [float(x) for x in sol], rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("Qx,Nx", [(4, 3), (16, 10), (80, 10)])
def test_gx_at_reference_state_is_the_weight(Qx, Nx):
    # at (u, T) = (0, p0^2) the truncation reproduces the quadrature weights exactly
    p = OracleProblem(Qx, 4, 8, Nx=Nx)
    g = p.gx(0.0, 1.0)
    np.testing.assert_allclose(g, np.concatenate([p.wx, p.wx]), rtol=1e-14, atol=0)


@pytest.mark.parametrize("Qy,Ny,u,T", [(4, 3, 0.05, 1.02), (7, 6, -0.3, 0.8), (12, 11, 0.5, 1.2),
                                       (20, 19, 0.25, 1.05)])
def test_gy_recovers_full_range_moments(Qy, Ny, u, T):
    p = OracleProblem(4, Qy, 8, Ny=Ny)
    g = p.gy(u, T)
    for l in range(Ny + 1):
        assert float(np.sum(g * p.zy ** l)) == pytest.approx(_full_moment(l, u, T), rel=1e-12, abs=1e-14)


def test_gy_at_reference_state_is_the_weight():
    p = OracleProblem(4, 8, 8)
    np.testing.assert_allclose(p.gy(0.0, 1.0), p.wy, rtol=1e-15)


def _mixture_state(p, comps):
    """phi, chi for a mixture of truncated Maxwellians: comps = [(weight, ux, uy, T)]."""
    phi = np.zeros((p.nv, p.ncell))
    for (a, ux, uy, T) in comps:
        f = a * np.outer(p.gx(ux, T), p.gy(uy, T)).reshape(-1)
        phi += f[:, None]
    chi = np.zeros_like(phi)
    for (a, ux, uy, T) in comps:
        f = a * np.outer(p.gx(ux, T), p.gy(uy, T)).reshape(-1)
        chi += T * f[:, None]
    return phi, chi


def test_moments_of_a_two_maxwellian_mixture_match_closed_form():
    # mixture of two Maxwellians: n, u, P_ij, T_zz, T and q follow in closed form
    p = OracleProblem(8, 8, 8, Nx=7, Ny=7)
    comps = [(0.6, 0.1, -0.2, 1.1), (0.4, -0.15, 0.3, 0.9)]
    phi, chi = _mixture_state(p, comps)
    m = p.moments(phi, chi)[:, 0]
    n = sum(a for a, *_ in comps)
    ux = sum(a * cx for a, cx, cy, T in comps) / n
    uy = sum(a * cy for a, cx, cy, T in comps) / n
    pxx = sum(a * (T + (cx - ux) ** 2) for a, cx, cy, T in comps)
    pyy = sum(a * (T + (cy - uy) ** 2) for a, cx, cy, T in comps)
    pxy = sum(a * (cx - ux) * (cy - uy) for a, cx, cy, T in comps)
    tzz = sum(a * T for a, cx, cy, T in comps)
    Tm = (pxx + pyy + tzz) / (3 * n)
    # q_x = 1/2 sum_k a_k < (xi_x^2 + xi_y^2 + xi_z^2) xi_x > with xi = c_k - u + thermal part
    qx = qy = 0.0
    for a, cx, cy, T in comps:
        dx, dy = cx - ux, cy - uy
        qx += 0.5 * a * (dx * (dx * dx + dy * dy) + dx * 5 * T)
        qy += 0.5 * a * (dy * (dx * dx + dy * dy) + dy * 5 * T)
    expect = [n, ux, uy, Tm, pxx, pxy, pyy, tzz, qx, qy]
    np.testing.assert_allclose(m, expect, rtol=1e-12, atol=1e-14)


def test_shakhov_target_conserves_and_relaxes_heat_flux_to_one_minus_Pr():
    # Sec. II: the Shakhov factor leaves n, u, T unchanged and gives the equilibrium part the
    # heat flux (1 - Pr) q; exact for the reduced pair once both truncations reach degree 6.
    p = OracleProblem(8, 8, 8, Nx=7, Ny=7, Pr=2.0 / 3.0)
    n, ux, uy, T, qx, qy = 1.07, 0.03, -0.12, 1.04, 0.021, -0.013
    tp, tc = p.collision_target(n, ux, uy, T, qx, qy)
    phi = np.repeat(tp[:, None], p.ncell, axis=1)
    chi = np.repeat(tc[:, None], p.ncell, axis=1)
    m = p.moments(phi, chi)[:, 0]
    assert m[0] == pytest.approx(n, rel=1e-13)
    assert m[1] == pytest.approx(ux, rel=1e-11)
    assert m[2] == pytest.approx(uy, rel=1e-12)
    assert m[3] == pytest.approx(T, rel=1e-13)
    assert m[5] == pytest.approx(0.0, abs=1e-14)
    assert m[8] == pytest.approx((1 - p.Pr) * qx, rel=1e-11)
    assert m[9] == pytest.approx((1 - p.Pr) * qy, rel=1e-11)


def test_shakhov_heat_flux_detects_wrong_constant():
    # the same moment with the -4/5 of S_phi replaced is far from (1 - Pr) q: the pin above
    # discriminates that constant (computed here with the oracle's own g tables)
    p = OracleProblem(8, 8, 8, Nx=7, Ny=7)
    n, T, qx = 1.0, 1.0, 0.02
    gx, gy = p.gx(0, T), p.gy(0, T)
    feq = n * np.outer(gx, gy).reshape(-1)
    xi2 = p.px ** 2 + p.py ** 2
    pref = (1 - p.Pr) / (n * T * T)
    wrong = feq * (1 + pref * (xi2 / (5 * T) - 3.0 / 5.0) * qx * p.px)
    chi = T * feq * (1 + pref * (xi2 / (5 * T) - 2.0 / 5.0) * qx * p.px)
    q = 0.5 * np.sum(xi2 * p.px * wrong + p.px * chi)
    assert abs(q - (1 - p.Pr) * qx) > 1e-3


@pytest.mark.parametrize("delta,omega", [(1.0, 0.7), (0.1, 0.66), (10.0, 0.5)])
def test_tau_reproduces_delta_and_viscosity_law(delta, omega):
    # equation (delta): delta = L P_ref/(mu(T_w) v_ref sqrt 2) with mu = tau P (Sec. II);
    # equation (mu): mu(T)/mu(T_w) = (T/T_w)^omega, with mu = tau n K_B T
    p = OracleProblem(4, 4, 8, delta=delta, omega=omega)
    mu_w = p.tau(1.0, 1.0) * 1.0 * 1.0
    assert 1.0 * 1.0 / (mu_w * 1.0 * math.sqrt(2)) == pytest.approx(delta, rel=1e-14)
    for n, T in [(0.9, 1.2), (1.3, 0.8)]:
        mu = p.tau(n, T) * n * T
        assert mu / mu_w == pytest.approx(T ** omega, rel=1e-14)


# ---- tabulated transport law, equations (mun) and (interp) -------------------------------------
POWER_TABLE_T = [0.5, 0.8, 1.0, 1.3, 2.0]


def _power_table(omega, Pr, c=3.7):
    return [(T, c * T ** omega, Pr) for T in POWER_TABLE_T]


def test_table_sampled_from_a_power_law_reproduces_it():
    # every interval's omega_n of (mun) is the sampled exponent, inside and outside the table
    omega, Pr = 0.7, 2.0 / 3.0
    a = OracleProblem(4, 4, 16, delta=0.8, omega=omega, Pr=Pr, stretch_A=0.9, uw=0.3)
    b = OracleProblem(4, 4, 16, delta=0.8, stretch_A=0.9, uw=0.3, visc_table=_power_table(omega, Pr))
    for T in (0.3, 0.5, 0.66, 0.8, 0.97, 1.0, 1.2, 1.3, 1.9, 2.0, 3.1):
        assert b.tau(1.1, T) == pytest.approx(a.tau(1.1, T), rel=1e-14)
        assert b.prandtl(T) == Pr
    pa, ca = a.init_state()
    pb, cb = b.init_state()
    a.step(pa, ca, 100)
    b.step(pb, cb, 100)
    assert np.max(np.abs(pa - pb)) <= 1e-13 * np.max(pa)


def _random_table(seed, N=6):
    rng = np.random.default_rng(seed)
    T = np.sort(rng.uniform(0.4, 2.5, N))
    mu = np.exp(rng.uniform(-0.5, 0.5, N)) * T ** 0.7
    Pr = rng.uniform(0.6, 0.75, N)
    return T, mu, Pr


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_table_law_passes_through_the_tabulated_values(seed):
    # mu^(n)(T_n) = mu_n and mu^(n)(T_{n+1}) = mu_{n+1}: with T_w placed on node k, eq. (tau) gives
    # tau n T / T_w = (mu(T)/mu_k) / (delta sqrt 2) / sqrt(T_w) at every node, from either side
    T, mu, Pr = _random_table(seed)
    k, delta = 2, 0.9
    p = OracleProblem(4, 4, 8, delta=delta, Tw=T[k], visc_table=list(zip(T, mu, Pr)))

    def ratio(Tq):
        return p.tau(1.0, Tq) * (Tq / T[k]) * delta * math.sqrt(2.0) * math.sqrt(T[k])

    for n in range(len(T)):
        assert ratio(T[n]) == pytest.approx(mu[n] / mu[k], rel=1e-13)
        for eps in (1e-12, -1e-12):  # continuity from both sides (|omega_n| stays below 1e3 here)
            assert ratio(T[n] * (1 + eps)) == pytest.approx(mu[n] / mu[k], rel=1e-9)
    # beyond the table the end intervals continue: (T/T_1)^omega_1 below, (T/T_N)^omega_{N-1} above
    om1 = math.log(mu[1] / mu[0]) / math.log(T[1] / T[0])
    omN = math.log(mu[-1] / mu[-2]) / math.log(T[-1] / T[-2])
    assert ratio(0.5 * T[0]) == pytest.approx(mu[0] * 0.5 ** om1 / mu[k], rel=1e-13)
    assert ratio(1.5 * T[-1]) == pytest.approx(mu[-1] * 1.5 ** omN / mu[k], rel=1e-13)


def test_table_prandtl_is_piecewise_constant_as_in_interp():
    # Pr_1 below T_2 (also below T_1), Pr_n on [T_n, T_{n+1}), Pr_N from T_N on
    T, mu, Pr = _random_table(5)
    p = OracleProblem(4, 4, 8, visc_table=list(zip(T, mu, Pr)))
    N = len(T)
    assert p.prandtl(0.5 * T[0]) == Pr[0]
    assert p.prandtl(T[0]) == Pr[0]
    assert p.prandtl(0.5 * (T[0] + T[1])) == Pr[0]
    for n in range(1, N - 1):
        assert p.prandtl(T[n]) == Pr[n]
        assert p.prandtl(0.5 * (T[n] + T[n + 1])) == Pr[n]
    assert p.prandtl(T[N - 1]) == Pr[N - 1]
    assert p.prandtl(2.0 * T[N - 1]) == Pr[N - 1]


def test_shakhov_target_uses_the_tabulated_prandtl_number():
    # the heat flux of the collision target is (1 - Pr(T)) q with Pr(T) from the table's interval
    T, mu, Pr = _random_table(7)
    p = OracleProblem(8, 8, 8, Nx=7, Ny=7, visc_table=list(zip(T, mu, Pr)))
    for Tc in (0.5 * (T[1] + T[2]), 0.5 * (T[3] + T[4])):
        n, qx, qy = 1.05, 0.02, -0.01
        tp, tc = p.collision_target(n, 0.01, -0.03, Tc, qx, qy)
        m = p.moments(np.repeat(tp[:, None], 8, axis=1), np.repeat(tc[:, None], 8, axis=1))[:, 0]
        pr = Pr[int(np.searchsorted(T, Tc, side="right")) - 1]
        assert m[8] == pytest.approx((1 - pr) * qx, rel=1e-10)
        assert m[9] == pytest.approx((1 - pr) * qy, rel=1e-10)

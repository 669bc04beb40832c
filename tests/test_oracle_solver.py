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

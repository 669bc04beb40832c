"""Pins of the oracle's diffuse-wall closure (Sec. III WENO-5 with eqs. diffuse and diffuse_nw; the
paper does not say how the stencil is closed at a wall) and of its steady-state residual norm.

- The ghosts of directions leaving through a wall are the quadratic through the three cells next to
  the wall: any quadratic (in the cell index) is reproduced exactly at the ghost positions, and
  directions entering from a wall see the wall population in their ghosts and on the wall face.
- The advection derivative of the cell next to a wall converges at second order on smooth data
  (ghost errors O(h^3) over a face difference divided by h); a linear extrapolation gives first
  order, a ghost shifted by one cell none.
- A second consistent closure (truncated WENO stencils, no ghost values read) gives the same shear
  stress as the grid is refined: the closure is a discretisation choice, not a change of the problem.
- The residual after one step is the J-weighted relative norm of the right-hand side to O(dt)."""
import math

import numpy as np
import pytest

from oracle.oracle import OracleProblem, weno5, weno5_sub


def test_truncated_weno_keeps_the_linear_weights_of_the_kept_stencils():
    rng = np.random.default_rng(5)
    for _ in range(20):
        v = rng.uniform(0.5, 1.5, 5)
        assert weno5_sub(*v, 7) == weno5(*v)
        # one stencil alone: its own candidate value, whatever the others hold
        a, b, c, d, e = v
        assert weno5_sub(a, b, c, d, e, 1) == pytest.approx((2 * a - 7 * b + 11 * c) / 6, rel=1e-14)
        assert weno5_sub(a, b, c, d, e, 4) == pytest.approx((2 * c + 5 * d - e) / 6, rel=1e-14)
        assert weno5_sub(a, b, c, d, 1e30, 3) == weno5_sub(a, b, c, d, -7.0, 3)
    # smooth data: two stencils with linear weights 0.1 and 0.6 renormalised (1/7, 6/7)
    x = np.linspace(0.0, 0.04, 5)
    f = 1.0 + 0.1 * x
    lin = (1 / 7) * (2 * f[0] - 7 * f[1] + 11 * f[2]) / 6 + (6 / 7) * (-f[1] + 5 * f[2] + 2 * f[3]) / 6
    assert weno5_sub(*f, 3) == pytest.approx(lin, rel=1e-12)


@pytest.mark.parametrize("half", [False, True])
def test_ghosts_reproduce_any_quadratic_at_the_wall(half):
    N = 12
    p = OracleProblem(4, 4, N, half_channel=half)
    rng = np.random.default_rng(7)
    s = np.arange(N, dtype=np.float64)
    for _ in range(5):
        c0, c1, c2 = rng.uniform(-1, 1, 3)
        q = lambda t: c0 + c1 * t + c2 * t * t  # noqa: E731
        f = q(s)
        wl, wr = 0.37, 0.61
        fm = rng.uniform(0.5, 1.5, N)
        # p_x > 0 leaves through the right wall: ghosts N, N+1, N+2 are the quadratic there
        e, F = p.row_faces(+0.8, f, wl, wr, fm if half else None)
        np.testing.assert_allclose(e[3 + N:], q(np.array([N, N + 1, N + 2], dtype=np.float64)), rtol=0, atol=1e-12)
        if half:  # the mirrored row of (-p_x, -p_y) continues the row left of x = 0
            np.testing.assert_array_equal(e[:3], fm[2::-1])
        else:  # the left wall's population enters: ghosts and the wall face
            np.testing.assert_array_equal(e[:3], [wl, wl, wl])
            assert F[0] == wl
        # p_x < 0 leaves through the left wall: ghosts -1, -2, -3 are the quadratic there
        e, F = p.row_faces(-0.8, f, wl, wr, fm if half else None)
        if not half:
            np.testing.assert_allclose(e[:3], q(np.array([-3, -2, -1], dtype=np.float64)), rtol=0, atol=1e-12)
        np.testing.assert_array_equal(e[3 + N:], [wr, wr, wr])
        assert F[N] == wr


@pytest.mark.parametrize("closure", [0, 1])
def test_near_wall_advection_derivative_converges_at_second_order(closure):
    # f smooth on [-1/2, 1/2]; the conservative difference (F_{s+1/2} - F_{s-1/2})/h at the cell next to
    # the wall that a direction leaves through, against f'(x_s)
    f = lambda x: np.exp(0.5 * np.sin(3.0 * x) + x)  # noqa: E731
    df = lambda x: f(x) * (1.5 * np.cos(3.0 * x) + 1.0)  # noqa: E731
    errs = {}
    for N in (32, 64, 128, 256):
        p = OracleProblem(4, 4, N, wall_closure=closure)
        x = p.x
        h = 1.0 / N
        _, F = p.row_faces(-1.0, f(x))
        e_left = abs((F[1] - F[0]) / h - df(x[0]))
        _, F = p.row_faces(+1.0, f(x))
        e_right = abs((F[N] - F[N - 1]) / h - df(x[N - 1]))
        errs[N] = (e_left, e_right)
    for side in (0, 1):
        orders = [math.log2(errs[n][side] / errs[2 * n][side]) for n in (32, 64, 128)]
        assert min(orders) > 1.8, (closure, side, orders, errs)
    # the interior is the fifth-order scheme: far from the walls the error is much smaller
    p = OracleProblem(4, 4, 256)
    _, F = p.row_faces(-1.0, f(p.x))
    mid = 128
    assert abs((F[mid + 1] - F[mid]) * 256 - df(p.x[mid])) < 1e-3 * errs[256][0]


def _steady_pi(N, closure, tol=1e-11):
    p = OracleProblem(4, 4, N, delta=1.0, uw=0.1, omega=0.7, wall_closure=closure)
    phi, chi = p.init_state()
    _, res = p.step(phi, chi, 200000, 200, tol)
    assert res < tol
    return p.Pi(p.moments(phi, chi))


@pytest.mark.slow
def test_the_two_wall_closures_agree_as_the_grid_is_refined():
    # measured: |Pi(BC-1) - Pi(BC-2)| = 7.1e-5, 1.75e-5, 4.3e-6 (and 1.1e-6 at 128 cells), both towards
    # Pi = 0.339141
    d = {}
    for N in (16, 32, 64):
        d[N] = (_steady_pi(N, 0), _steady_pi(N, 1))
    diff = {N: abs(a - b) for N, (a, b) in d.items()}
    orders = [math.log2(diff[n] / diff[2 * n]) for n in (16, 32)]
    assert min(orders) > 1.5, (d, orders)
    assert diff[64] < 2e-5 * d[64][0]


@pytest.mark.parametrize("lts", [0.0, 64.0])
def test_residual_is_the_relative_norm_of_the_right_hand_side(lts):
    rng = np.random.default_rng(11)
    kw = dict(delta=1.0, uw=0.2, stretch_A=0.9, local_dt_cap=lts)
    p0 = OracleProblem(4, 4, 32, **kw)
    phi0, chi0 = p0.init_state()
    phi0 = phi0 * (1 + 0.05 * rng.uniform(-1, 1, phi0.shape))
    chi0 = chi0 * (1 + 0.05 * rng.uniform(-1, 1, chi0.shape))
    dp, dc, _ = p0.rhs(phi0, chi0)
    J = p0.J[None, :]
    r0 = math.sqrt(np.sum(J * (dp ** 2 + dc ** 2))) / math.sqrt(np.sum(J * (phi0 ** 2 + chi0 ** 2)))
    dev = []
    for scale in (1.0, 0.5, 0.25):
        p = OracleProblem(4, 4, 32, dt=p0.dt * scale, **kw)
        phi, chi = phi0.copy(), chi0.copy()
        _, r = p.step(phi, chi, 1, 1, 0.0)
        dev.append(abs(r - r0) / r0)
    # first order in dt: the deviation halves with dt
    assert 1.6 < dev[0] / dev[1] < 2.4 and 1.6 < dev[1] / dev[2] < 2.4, dev
    assert dev[2] < 0.05

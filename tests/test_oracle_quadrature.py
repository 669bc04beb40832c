"""Pins for the oracle's quadrature tables (paper Sec. III), checked against brute-force
integration, the paper's closed-form weights and an independent library routine."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import quadrature as quad


@pytest.mark.parametrize("k", range(0, 9))
def test_half_range_moment_closed_form_matches_brute_force(k):
    # mu_k = int_0^inf z^k e^{-z^2/2}/sqrt(2 pi) dz, checked by numerical integration
    with mp.workdps(40):
        brute = mp.quad(lambda z: z ** k * mp.exp(-z * z / 2) / mp.sqrt(2 * mp.pi), [0, mp.inf])
        assert abs(brute - quad.half_range_moment(k)) < mp.mpf(10) ** -30 * abs(brute)


@pytest.mark.parametrize("Q", [3, 4, 7, 8, 16, 32])
def test_half_range_rule_exact_below_degree_2Q(Q):
    # Sec. III: equality of the half-range quadrature holds for s < 2Q
    r = quad.half_range_rule(Q)
    with mp.workdps(r.dps):
        for s in range(2 * Q):
            approx = sum(w * z ** s for w, z in zip(r.weights, r.nodes))
            exact = quad.half_range_moment(s)
            assert abs(approx - exact) < mp.mpf(10) ** -50 * exact, s
        # ... and fails at s = 2Q (checked where the deviation is far above round-off)
        if Q <= 8:
            approx = sum(w * z ** (2 * Q) for w, z in zip(r.weights, r.nodes))
            exact = quad.half_range_moment(2 * Q)
            assert abs(approx - exact) > mp.mpf(10) ** -8 * exact


@pytest.mark.parametrize("Q", [3, 4, 7, 8, 16, 32, 50])
def test_christoffel_weights_match_paper_closed_form(Q):
    # Sec. III weight formula w_i = p_i a_{Q-1}^2 / (h_{Q-1}^2(p_i) [p_i + p0 h_Q^2(0)/sqrt(2 pi)])
    r = quad.half_range_rule(Q)
    with mp.workdps(r.dps):
        for i in range(Q):
            paper = quad.paper_half_range_weight(r, i)
            assert abs(paper - r.weights[i]) < mp.mpf(10) ** -40 * r.weights[i]


@pytest.mark.parametrize("Q", [4, 7])
def test_half_range_polynomials_orthonormal_by_brute_force(Q):
    # reading: h_l orthonormal under e^{-z^2/2}/sqrt(2 pi) on [0, inf); checked with mp.quad
    r = quad.half_range_rule(Q)
    with mp.workdps(30):
        for l in range(4):
            for k in range(l, 4):
                val = mp.quad(lambda z: r.eval_h(l, z) * r.eval_h(k, z) * mp.exp(-z * z / 2)
                              / mp.sqrt(2 * mp.pi), [0, 2, 6, mp.inf])
                assert abs(val - (1 if l == k else 0)) < 1e-20


@pytest.mark.parametrize("Q", [4, 8])
def test_half_range_nodes_are_roots_and_positive(Q):
    r = quad.half_range_rule(Q)
    z = r.nodes_f64()
    assert np.all(z > 0) and np.all(np.diff(z) > 0)
    assert abs(float(sum(r.weights)) - 0.5) < 1e-15
    with mp.workdps(r.dps):
        for zi in r.nodes:
            assert abs(r.eval_h(Q, zi)) < mp.mpf(10) ** -40


@pytest.mark.parametrize("Q", [3, 4, 7, 8, 12, 20])
def test_full_range_rule_matches_numpy_hermegauss(Q):
    # paper weights w_j = Q!/He_{Q+1}(z_j)^2 against numpy's Gauss-Hermite-E rule / sqrt(2 pi)
    x, w = np.polynomial.hermite_e.hermegauss(Q)
    fr = quad.full_range_rule(Q)
    np.testing.assert_allclose(fr.nodes_f64(), x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(fr.weights_f64(), w / math.sqrt(2 * math.pi), rtol=1e-11)
    assert abs(sum(fr.weights_f64()) - 1.0) < 1e-14


@pytest.mark.parametrize("Q", [4, 7, 20])
def test_full_range_rule_exact_below_degree_2Q(Q):
    fr = quad.full_range_rule(Q)
    with mp.workdps(fr.dps):
        for s in range(2 * Q):
            approx = sum(w * z ** s for w, z in zip(fr.weights, fr.nodes))
            exact = mp.mpf(0) if s % 2 else mp.fac2(s - 1)
            assert abs(approx - exact) < mp.mpf(10) ** -40 * max(1, exact)


def test_velocity_counts_printed_in_paper():
    # Sec. IV / conclusion: HHLB(6;7) x HLB(6;7) has 98 velocities, HHLB(10;16) x HLB(6;7) has 224
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_velocity_counts.json")
    with open(path) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        hr = quad.half_range_rule(c["Qx"])
        fr = quad.full_range_rule(c["Qy"])
        assert 2 * len(hr.nodes) * len(fr.nodes) == c["velocities"]

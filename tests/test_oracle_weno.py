"""Pins for the oracle's WENO-5 face reconstruction (Jiang & Shu 1996, named in Sec. III).

The candidate values, smoothness indicators and linear weights are rebuilt here from their
definitions (quadratics matching cell averages, integrals of squared derivatives, and the
condition that the linear combination reproduces the five-cell reconstruction), not retyped."""
import numpy as np
import pytest

from oracle.oracle import weno5

EPS = 1e-6


def _quadratic_from_averages(centres, avgs):
    # p(x) = a + b x + c x^2 with mean over [m - 1/2, m + 1/2] equal to avgs
    M = np.array([[1.0, m, m * m + 1.0 / 12.0] for m in centres])
    return np.linalg.solve(M, np.asarray(avgs, dtype=float))


def _quartic_face_value(avgs):
    centres = [-2, -1, 0, 1, 2]
    M = np.array([[((m + 0.5) ** (k + 1) - (m - 0.5) ** (k + 1)) / (k + 1) for k in range(5)]
                  for m in centres])
    coef = np.linalg.solve(M, np.asarray(avgs, dtype=float))
    return sum(c * 0.5 ** k for k, c in enumerate(coef))


def _candidates_and_indicators(vals):
    qs, betas = [], []
    for k in range(3):
        centres = [-2 + k, -1 + k, k]
        a, b, c = _quadratic_from_averages(centres, vals[k:k + 3])
        qs.append(a + 0.5 * b + 0.25 * c)
        # beta = int_{-1/2}^{1/2} (p')^2 + (p'')^2 dx with p' = b + 2 c x, p'' = 2 c
        betas.append(b * b + c * c / 3.0 + 4.0 * c * c)
    return np.array(qs), np.array(betas)


def _linear_weights():
    rng = np.random.default_rng(3)
    rows, rhs = [], []
    for _ in range(3):
        v = rng.normal(size=5)
        q, _ = _candidates_and_indicators(v)
        rows.append(q)
        rhs.append(_quartic_face_value(v))
    return np.linalg.solve(np.array(rows), np.array(rhs))


def _reference_weno(vals):
    d = _linear_weights()
    q, beta = _candidates_and_indicators(vals)
    alpha = d / (EPS + beta) ** 2
    return float(np.sum(alpha * q) / np.sum(alpha))


def test_linear_weights_are_one_tenth_six_tenths_three_tenths():
    np.testing.assert_allclose(_linear_weights(), [0.1, 0.6, 0.3], rtol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_weno5_matches_definition_on_random_data(seed):
    rng = np.random.default_rng(seed)
    scale = [1e-4, 1e-2, 1.0][seed % 3]
    vals = scale * rng.normal(size=5) + rng.uniform(0, 1)
    assert weno5(*vals) == pytest.approx(_reference_weno(vals), rel=1e-13, abs=1e-16)


def test_weno5_small_amplitude_reduces_to_fifth_order_linear_scheme():
    rng = np.random.default_rng(7)
    vals = 1e-9 * rng.normal(size=5)
    linear = np.dot([2, -13, 47, 27, -3], vals) / 60.0
    assert weno5(*vals) == pytest.approx(linear, rel=1e-9)


def test_weno5_is_essentially_non_oscillatory_at_a_jump():
    # a step between the upwind cell and the next: the value stays on the upwind side
    v = weno5(0.0, 0.0, 0.0, 1.0, 1.0)
    assert abs(v) < 1e-6


@pytest.mark.parametrize("direction", [+1, -1])
def test_flux_difference_converges_at_fifth_order_on_smooth_data(direction):
    # (F_{i+1/2} - F_{i-1/2})/h -> f'(x) with error O(h^5) away from critical points
    f = lambda x: np.exp(2 * x) + 0.5 * x
    df = lambda x: 2 * np.exp(2 * x) + 0.5
    errs = []
    for h in (0.08, 0.04, 0.02):
        x0 = 0.3
        cells = x0 + h * np.arange(-4, 5)   # index 4 is x0

        def face(k):  # face between cells k-1 and k (array indices)
            if direction > 0:
                return weno5(*f(cells[k - 3:k + 2]))
            return weno5(*f(cells[k - 2:k + 3])[::-1])
        d = (face(5) - face(4)) / h
        errs.append(abs(d - df(x0)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 4.5), rates

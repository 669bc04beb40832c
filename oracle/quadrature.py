"""Oracle quadrature tables, in arbitrary precision (mpmath).

TEST INFRASTRUCTURE. This module belongs to the CPU oracle: only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it.  The GPU
product path has its own, independent quadrature code.

What is computed (paper, Sec. III "Mixed quadrature lattice Boltzmann models"):

* Half-range Gauss-Hermite rule on [0, inf) for the weight
  omega(z) = exp(-z^2/2)/sqrt(2 pi) (reference momentum p0 = 1).  The nodes are the
  roots of the half-range Hermite polynomial h_Q and the rule is exact for
  monomials z^s with s < 2Q (half-range quadrature equation).  The velocity set
  on the x axis is p_i = z_i and p_{i+Q} = -z_i with equal weights.
* Full-range Gauss-Hermite rule for the same weight on (-inf, inf): nodes are
  the roots of the probabilists' Hermite polynomial He_Q, weights
  Q!/He_{Q+1}(z_j)^2 (full-range quadrature equation and the weight formula
  that follows it).
* The table Phi_{s,i} = sum_{l=s}^{N} h_{l,s} h_l(z_i) used by the half-range
  polynomial truncation of the equilibrium (equation for g_{x,i}).

Readings (the paper leaves these implicit):
* h_l is taken ORTHONORMAL under omega on [0, inf); h_{l,s} is the coefficient
  of z^s in h_l; a_l = h_{l+1,l+1}/h_{l,l}.
* The recurrence coefficients are obtained from the exact moments of omega by
  the Chebyshev algorithm (Gautschi, "Orthogonal Polynomials: Computation and
  Approximation", 2004, Sec. 2.1.7), carried out with enough digits that the
  ill-conditioning of the moment map is harmless; nodes by Newton iteration on
  the three-term recurrence; weights by the Christoffel-number formula
  w_i = 1/sum_{l<Q} h_l(z_i)^2.  The paper's own closed form for w_i is kept
  separately (``paper_half_range_weight``) so that the tests can check one
  against the other.
"""
from __future__ import annotations

import functools
import math

import mpmath as mp
import numpy as np

__all__ = [
    "half_range_moment",
    "HalfRangeRule",
    "half_range_rule",
    "paper_half_range_weight",
    "FullRangeRule",
    "full_range_rule",
    "phi_table",
    "split_hi_lo",
]


def _dps_for(Q: int) -> int:
    # The moment -> recurrence map loses roughly one digit per unit of Q for this
    # weight; 4 digits per unit plus a margin of 80 keeps >= 60 correct digits.
    return 80 + 4 * Q


def half_range_moment(k: int) -> mp.mpf:
    """mu_k = int_0^inf z^k exp(-z^2/2)/sqrt(2 pi) dz = 2^((k-1)/2) Gamma((k+1)/2)/sqrt(2 pi)."""
    return mp.power(2, mp.mpf(k - 1) / 2) * mp.gamma(mp.mpf(k + 1) / 2) / mp.sqrt(2 * mp.pi)


def _chebyshev_algorithm(mom, n):
    """Monic recurrence pi_{k+1} = (z - alpha_k) pi_k - beta_k pi_{k-1} from moments mom[0..2n-1]."""
    alpha = [mp.mpf(0)] * n
    beta = [mp.mpf(0)] * n
    sig_prev = [mp.mpf(0)] * (2 * n)           # sigma_{-1, l}
    sig = [mom[l] for l in range(2 * n)]        # sigma_{0, l}
    alpha[0] = mom[1] / mom[0]
    beta[0] = mom[0]
    for k in range(1, n):
        sig_new = [mp.mpf(0)] * (2 * n)
        for l in range(k, 2 * n - k):
            sig_new[l] = sig[l + 1] - alpha[k - 1] * sig[l] - beta[k - 1] * sig_prev[l]
        alpha[k] = sig_new[k + 1] / sig_new[k] - sig[k] / sig[k - 1]
        beta[k] = sig_new[k] / sig[k - 1]
        sig_prev, sig = sig, sig_new
    return alpha, beta


class HalfRangeRule:
    """Half-range Gauss-Hermite rule of order Q (positive semi-axis only)."""

    def __init__(self, Q: int):
        if Q < 1:
            raise ValueError("Q must be >= 1")
        self.Q = Q
        self.dps = _dps_for(Q)
        with mp.workdps(self.dps):
            mom = [half_range_moment(k) for k in range(2 * Q + 2)]
            self.alpha, self.beta = _chebyshev_algorithm(mom, Q + 1)
            # orthonormal monomial coefficients coef[l][s] = h_{l,s}, l = 0..Q
            self.coef = self._orthonormal_coefficients(Q)
            self.nodes = self._nodes()
            self.weights = [1 / sum(self.eval_h(l, z) ** 2 for l in range(Q)) for z in self.nodes]

    # --- orthonormal polynomials ---------------------------------------------------------
    def _orthonormal_coefficients(self, L):
        # monic pi_l via the recurrence, then h_l = pi_l / sqrt(beta_0 ... beta_l)
        monic = [[mp.mpf(1)], [-self.alpha[0], mp.mpf(1)]]
        for l in range(1, L):
            a, b = self.alpha[l], self.beta[l]
            nxt = [mp.mpf(0)] * (l + 2)
            for s, c in enumerate(monic[l]):
                nxt[s + 1] += c
                nxt[s] -= a * c
            for s, c in enumerate(monic[l - 1]):
                nxt[s] -= b * c
            monic.append(nxt)
        out = []
        norm2 = mp.mpf(1)
        for l in range(L + 1):
            norm2 *= self.beta[l]
            inv = 1 / mp.sqrt(norm2)
            out.append([c * inv for c in monic[l]])
        return out

    def eval_h(self, l: int, z) -> mp.mpf:
        """h_l(z) by Horner on the monomial coefficients (exact-precision arithmetic)."""
        acc = mp.mpf(0)
        for c in reversed(self.coef[l]):
            acc = acc * z + c
        return acc

    def _eval_monic(self, n: int, z):
        p_prev, p = mp.mpf(0), mp.mpf(1)
        dp_prev, dp = mp.mpf(0), mp.mpf(0)
        for k in range(n):
            p_next = (z - self.alpha[k]) * p - (self.beta[k] * p_prev if k > 0 else 0)
            dp_next = p + (z - self.alpha[k]) * dp - (self.beta[k] * dp_prev if k > 0 else 0)
            p_prev, p = p, p_next
            dp_prev, dp = dp, dp_next
        return p, dp

    def _nodes(self):
        Q = self.Q
        # float64 starting values from the Jacobi matrix, then Newton at full precision
        a = np.array([float(x) for x in self.alpha[:Q]])
        b = np.array([math.sqrt(float(x)) for x in self.beta[1:Q]])
        jac = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        guess = np.sort(np.linalg.eigvalsh(jac))
        roots = []
        for g in guess:
            z = mp.mpf(float(g))
            for _ in range(200):
                p, dp = self._eval_monic(Q, z)
                step = p / dp
                z -= step
                if abs(step) < mp.mpf(10) ** (-(self.dps - 10)) * max(1, abs(z)):
                    break
            roots.append(z)
        return roots

    # --- convenience -------------------------------------------------------------------
    def a(self, l: int) -> mp.mpf:
        return self.coef[l + 1][l + 1] / self.coef[l][l]

    def nodes_f64(self) -> np.ndarray:
        return np.array([float(z) for z in self.nodes])

    def weights_f64(self) -> np.ndarray:
        return np.array([float(w) for w in self.weights])


@functools.lru_cache(maxsize=None)
def half_range_rule(Q: int) -> HalfRangeRule:
    return HalfRangeRule(Q)


def paper_half_range_weight(rule: HalfRangeRule, i: int) -> mp.mpf:
    """Closed form of the half-range weight printed in Sec. III (p0 = 1):

    w_i = z_i a_{Q-1}^2 / ( h_{Q-1}(z_i)^2 [ z_i + h_Q(0)^2/sqrt(2 pi) ] ).
    """
    Q = rule.Q
    with mp.workdps(rule.dps):
        z = rule.nodes[i]
        aq = rule.a(Q - 1)
        hq0 = rule.coef[Q][0]
        return z * aq ** 2 / (rule.eval_h(Q - 1, z) ** 2 * (z + hq0 ** 2 / mp.sqrt(2 * mp.pi)))


class FullRangeRule:
    """Full-range Gauss-Hermite rule of order Q, weights normalised to sum 1."""

    def __init__(self, Q: int):
        self.Q = Q
        self.dps = 60 + 2 * Q
        with mp.workdps(self.dps):
            guess = np.sort(np.polynomial.hermite_e.hermeroots([0] * Q + [1]))
            self.nodes = []
            for g in guess:
                z = mp.mpf(float(g))
                for _ in range(200):
                    h, dh = self.eval_he(Q, z), Q * self.eval_he(Q - 1, z)
                    step = h / dh
                    z -= step
                    if abs(step) < mp.mpf(10) ** (-(self.dps - 10)) * max(1, abs(z)):
                        break
                self.nodes.append(z)
            # paper: w_j = Q!/He_{Q+1}(z_j)^2
            self.weights = [mp.factorial(Q) / self.eval_he(Q + 1, z) ** 2 for z in self.nodes]

    @staticmethod
    def eval_he(n: int, z):
        """Probabilists' Hermite polynomial He_n(z) (He_{n+1} = z He_n - n He_{n-1})."""
        p_prev, p = mp.mpf(0), mp.mpf(1)
        for k in range(n):
            p_prev, p = p, z * p - k * p_prev
        return p

    def nodes_f64(self) -> np.ndarray:
        return np.array([float(z) for z in self.nodes])

    def weights_f64(self) -> np.ndarray:
        return np.array([float(w) for w in self.weights])


@functools.lru_cache(maxsize=None)
def full_range_rule(Q: int) -> FullRangeRule:
    return FullRangeRule(Q)


@functools.lru_cache(maxsize=None)
def phi_table(Q: int, N: int):
    """Phi_{s,i} = sum_{l=s}^{N} h_{l,s} h_l(z_i) for s = 0..N, i = 0..Q-1 (mpf, [N+1][Q])."""
    if not 0 <= N <= Q:
        raise ValueError("expansion order N must satisfy 0 <= N <= Q")
    rule = half_range_rule(Q)
    with mp.workdps(rule.dps):
        hz = [[rule.eval_h(l, z) for z in rule.nodes] for l in range(N + 1)]
        return [[sum(rule.coef[l][s] * hz[l][i] for l in range(s, N + 1)) for i in range(Q)]
                for s in range(N + 1)]


def split_hi_lo(values) -> tuple[np.ndarray, np.ndarray]:
    """Split mpf values into float64 hi + lo with hi + lo equal to the value to ~32 digits."""
    hi = np.array([float(v) for v in values])
    lo = np.array([float(v - mp.mpf(h)) for v, h in zip(values, hi)])
    return hi, lo

"""Workload definitions and seeded draws (no method arithmetic).

Nondimensional units throughout: m = K_B = L = n_ref = 1, wall temperature T_w = 1, Pr = 2/3.
Expansion orders default to N_x = min(Q_x - 1, 10) and N_y = Q_y - 1.
"""
from __future__ import annotations

import numpy as np

__all__ = ["SINGLE_CASES", "case", "batch_draws", "poisson_arrivals", "perturb", "steady_calibration_draws"]

# The single-instance workloads (plain and mixed-precision).  A = 0 means a uniform grid.
SINGLE_CASES = {
    "couette_nx32_q4x4_fp64": dict(Qx=4, Qy=4, ncell=32, stretch_A=0.0, delta=1.0, uw=0.05,
                                   Tw=1.0, Pr=2.0 / 3.0, omega=0.7),
    "couette_nx512_q16x8": dict(Qx=16, Qy=8, ncell=512, stretch_A=0.9, delta=0.1, uw=0.2,
                                Tw=1.0, Pr=2.0 / 3.0, omega=0.66),
    "couette_nx2048_q80x20": dict(Qx=80, Qy=20, ncell=2048, stretch_A=0.9, delta=0.01, uw=0.5,
                                  Tw=1.0, Pr=2.0 / 3.0, omega=0.7),
}


def case(name: str, **overrides) -> dict:
    d = dict(SINGLE_CASES[name])
    d.update(overrides)
    return d


def batch_draws(n: int, seed: int = 0, nx_choices=(64, 128, 256, 512, 1024), qx_choices=(4, 8, 16, 32),
                qy_choices=(4, 8, 12), stretch_A: float = 0.9) -> list[dict]:
    """Ragged instance parameters drawn in a fixed order per instance:
    delta = 10^U(-2, 2), u_w ~ U(0.01, 0.5), omega ~ U(0.5, 1.0), Nx, Qx, Qy uniform over the choices."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        delta = float(10.0 ** rng.uniform(-2.0, 2.0))
        uw = float(rng.uniform(0.01, 0.5))
        omega = float(rng.uniform(0.5, 1.0))
        ncell = int(rng.choice(nx_choices))
        Qx = int(rng.choice(qx_choices))
        Qy = int(rng.choice(qy_choices))
        out.append(dict(Qx=Qx, Qy=Qy, ncell=ncell, stretch_A=stretch_A, delta=delta, uw=uw,
                        Tw=1.0, Pr=2.0 / 3.0, omega=omega, seed=seed * 1000003 + k))
    return out


def poisson_arrivals(n: int, rate: float, seed: int = 2) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def perturb(arr: np.ndarray, amp: float, seed: int) -> np.ndarray:
    """Multiply an array elementwise by (1 + amp * U(-1, 1)), seeded."""
    rng = np.random.default_rng(seed)
    return arr * (1.0 + amp * rng.uniform(-1.0, 1.0, size=arr.shape))


def steady_calibration_draws(n: int = 8, seed: int = 5) -> list[dict]:
    """Small solves drawn from the serving workload's parameter ranges, at sizes whose steady states the
    FP64 oracle reaches in minutes: delta = 10^U(-1, 2) (the serving range starts at 10^-2, whose
    strongly rarefied solves take the oracle hours), u_w ~ U(0.01, 0.5), omega ~ U(0.5, 1.0),
    Nx in {32, 64}, Qx in {4, 8}, Qy in {4, 8}; A = 0.9, T_w = 1, Pr = 2/3."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        delta = float(10.0 ** rng.uniform(-1.0, 2.0))
        uw = float(rng.uniform(0.01, 0.5))
        omega = float(rng.uniform(0.5, 1.0))
        ncell = int(rng.choice((32, 64)))
        Qx = int(rng.choice((4, 8)))
        Qy = int(rng.choice((4, 8)))
        out.append(dict(Qx=Qx, Qy=Qy, ncell=ncell, stretch_A=0.9, delta=delta, uw=uw, Tw=1.0, Pr=2.0 / 3.0,
                        omega=omega, seed=seed * 1000003 + k))
    return out

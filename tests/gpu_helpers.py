"""Shared helpers of the GPU tests: build a GPU case and an oracle case from the same parameters."""
import sys

import numpy as np


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def make_pair(Qx, Qy, ncell, *, stretch_A=0.0, delta=1.0, uw=0.05, Tw=1.0, Pr=2.0 / 3.0, omega=0.7,
              precision=0, rounding=0, dt=0.0, cfl=0.5, seed=0, half_channel=False):
    """(gpu_case, oracle_problem) sharing dt; the oracle picks dt by the same rule when dt <= 0."""
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    orc = OracleProblem(Qx, Qy, ncell, stretch_A=stretch_A, delta=delta, uw=uw, Tw=Tw, Pr=Pr, omega=omega,
                        dt=(dt if dt > 0 else None), cfl=cfl, collisionless=(delta == 0.0),
                        half_channel=half_channel)
    q = hrlb.Quadrature(Qx, Qy, orc.Nx, orc.Ny)
    params = hrlb.make_params(delta=delta, uw=uw, ncell=ncell, stretch_A=stretch_A, Tw=Tw, Pr=Pr, omega=omega,
                              precision=precision, rounding=rounding, cfl=cfl, dt=orc.dt, seed=seed,
                              half_channel=int(half_channel))
    case = hrlb.Case(q, params)
    case._quad_ref = q
    return case, orc


def rel_state_err(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| over the whole array."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def field_errs(f_gpu: np.ndarray, f_orc: np.ndarray):
    """Per-field max error relative to the larger of the field's own max magnitude and its natural
    scale (n_ref, sqrt(T_w), T_w, n_ref T_w, n_ref T_w^(3/2): all 1 in the solver's units)."""
    out = []
    for k in range(10):
        scale = max(np.max(np.abs(f_orc[k])), 1.0)
        out.append(float(np.max(np.abs(f_gpu[k] - f_orc[k])) / scale))
    return np.array(out)


def pxy_err(f_gpu: np.ndarray, f_orc: np.ndarray) -> float:
    """Shear stress error relative to its own magnitude (the headline quantity)."""
    return float(np.max(np.abs(f_gpu[5] - f_orc[5])) / np.max(np.abs(f_orc[5])))

"""Shared helpers of the GPU tests: build a GPU case and an oracle case from the same parameters,
and the error measures of the parity tests."""
import sys

import numpy as np

# populations are compared one by one, relative to their own value, above this fraction of the
# largest population of their distribution (the Gauss-Hermite tails reach 1e-30 and below, where a
# 1e-6 absolute WENO epsilon and FP32 subnormals make a relative comparison meaningless)
POP_FLOOR = 1e-2


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def make_pair(Qx, Qy, ncell, *, stretch_A=0.0, delta=1.0, uw=0.05, Tw=1.0, Pr=2.0 / 3.0, omega=0.7,
              precision=0, rounding=0, dt=0.0, cfl=0.5, seed=0, half_channel=False, Nx=None, Ny=None, path=1):
    """(gpu_case, oracle_problem) sharing dt; the oracle picks dt by the same rule when dt <= 0.  path: the
    GPU case's kernel path (default the tiled kernels; the small-case path has tests of its own)."""
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    orc = OracleProblem(Qx, Qy, ncell, Nx=Nx, Ny=Ny, stretch_A=stretch_A, delta=delta, uw=uw, Tw=Tw, Pr=Pr,
                        omega=omega, dt=(dt if dt > 0 else None), cfl=cfl, collisionless=(delta == 0.0),
                        half_channel=half_channel)
    q = hrlb.Quadrature(Qx, Qy, orc.Nx, orc.Ny)
    params = hrlb.make_params(delta=delta, uw=uw, ncell=ncell, stretch_A=stretch_A, Tw=Tw, Pr=Pr, omega=omega,
                              precision=precision, rounding=rounding, cfl=cfl, dt=orc.dt, seed=seed,
                              half_channel=int(half_channel), kernel_path=path)
    case = hrlb.Case(q, params)
    case._quad_ref = q
    return case, orc


def rel_state_err(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| over the whole array."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel_pop_err(a: np.ndarray, b: np.ndarray, floor: float = POP_FLOOR) -> float:
    """max over populations |a - b| / |b|, over the populations with |b| >= floor * max |b|."""
    b = np.asarray(b)
    keep = np.abs(b) >= floor * np.max(np.abs(b))
    return float(np.max(np.abs(a[keep] - b[keep]) / np.abs(b[keep])))


def state_errs(st: np.ndarray, phi: np.ndarray, chi: np.ndarray):
    """(max-norm error relative to the largest population, largest per-population relative error)."""
    e_max = max(rel_state_err(st[0], phi), rel_state_err(st[1], chi))
    e_pop = max(rel_pop_err(st[0], phi), rel_pop_err(st[1], chi))
    return e_max, e_pop


def term_scales(f_ref: np.ndarray) -> np.ndarray:
    """Per field, the size of the terms whose sum over the velocity set the field is, for a local
    Maxwellian with the reference's n and T: a floating-point sum of terms of size S carries
    errors of order eps S whatever its value, so a field much smaller than its terms (u_x, u_y,
    P_xy, q_x, q_y in a near-equilibrium flow) cannot be compared with two independent codes
    relative to itself.  With th = sqrt(2T/pi) the mean |xi_i| of a Maxwellian:
    n: n; u_i: th (sum |p_i| phi / n); T, P_xx, P_yy, T_zz: the field itself (positive terms);
    P_xy: 2 n T / pi (sum |xi_x xi_y| phi); q_i: 2 th n T (1/2 sum (|xi|^2 |xi_i| phi + |xi_i| chi))."""
    n, T = np.abs(f_ref[0]), np.abs(f_ref[3])
    th = np.sqrt(2.0 * T / np.pi)
    terms = [n, th, th, T, np.abs(f_ref[4]), 2.0 * n * T / np.pi, np.abs(f_ref[6]), np.abs(f_ref[7]),
             2.0 * th * n * T, 2.0 * th * n * T]
    return np.array([float(np.max(t)) for t in terms])


def field_errs(f_gpu: np.ndarray, f_ref: np.ndarray):
    """Per-field max error relative to the larger of the field's own largest magnitude and the size
    of its terms (term_scales)."""
    sc = term_scales(f_ref)
    out = []
    for k in range(10):
        scale = max(float(np.max(np.abs(f_ref[k]))), sc[k])
        out.append(float(np.max(np.abs(f_gpu[k] - f_ref[k])) / scale))
    return np.array(out)


# the fields compared relative to their own magnitude as well: the headline shear stress and the
# profiles the flow is read from (density, velocity along the walls, temperature)
OWN_FIELDS = (0, 2, 3, 5)


def own_errs(f_gpu: np.ndarray, f_ref: np.ndarray) -> np.ndarray:
    """max |error| / max |field| for n, u_y, T, P_xy (0 for a field that is zero everywhere)."""
    out = []
    for k in OWN_FIELDS:
        m = float(np.max(np.abs(f_ref[k])))
        out.append(float(np.max(np.abs(f_gpu[k] - f_ref[k])) / m) if m > 0 else 0.0)
    return np.array(out)


def pxy_err(f_gpu: np.ndarray, f_orc: np.ndarray) -> float:
    """Shear stress error relative to its own magnitude (the headline quantity)."""
    return float(np.max(np.abs(f_gpu[5] - f_orc[5])) / np.max(np.abs(f_orc[5])))


def fmt_errs(e) -> str:
    names = ("n", "ux", "uy", "T", "Pxx", "Pxy", "Pyy", "Tzz", "qx", "qy")
    return " ".join(f"{n}={v:.1e}" for n, v in zip(names, e))


def fmt_own(e) -> str:
    return " ".join(f"{n}={v:.1e}" for n, v in zip(("n", "uy", "T", "Pxy"), e))


def moment_errs(f_gpu: np.ndarray, f_ref: np.ndarray, tol: float, label: str = "") -> bool:
    """Prints and checks both measures: every field (field_errs) and n, u_y, T, P_xy against their own
    magnitude (own_errs), all below tol."""
    ef, eo = field_errs(f_gpu, f_ref), own_errs(f_gpu, f_ref)
    say(f"   {label}fields {fmt_errs(ef)}; own {fmt_own(eo)}")
    return bool(np.all(ef < tol) and np.all(eo < tol))


def pop_profile(st: np.ndarray, phi: np.ndarray, chi: np.ndarray) -> str:
    """Per-population relative error above several magnitude floors (diagnostic output)."""
    out = []
    for fl in (1e-2, 1e-4, 1e-6, 1e-9, 1e-12):
        e = max(rel_pop_err(st[0], phi, fl), rel_pop_err(st[1], chi, fl))
        out.append(f"{fl:.0e}:{e:.1e}")
    return " ".join(out)


def parity(st: np.ndarray, phi: np.ndarray, chi: np.ndarray, f_gpu: np.ndarray, f_orc: np.ndarray, tol: float,
           label: str = "", pop_floor: float = POP_FLOOR) -> bool:
    """Full parity check of a GPU state and its moments against the oracle's: the state in the
    max-norm and population by population (above pop_floor), and the moments (moment_errs)."""
    e_max = max(rel_state_err(st[0], phi), rel_state_err(st[1], chi))
    e_pop = max(rel_pop_err(st[0], phi, pop_floor), rel_pop_err(st[1], chi, pop_floor))
    say(f"   {label}state err {e_max:.3e}, per-population (>= {pop_floor:.0e} max) {e_pop:.3e} "
        f"[{pop_profile(st, phi, chi)}]")
    ok_m = moment_errs(f_gpu, f_orc, tol, label)
    return bool(e_max < tol and e_pop < tol and ok_m)

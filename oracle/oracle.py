"""Python front end of the CPU oracle (ctypes over hrlb_oracle.c).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the GPU library.

``OracleProblem`` gathers one Couette case (paper, Secs. II-III): quadrature orders
HHLB(Nx;Qx) x HLB(Ny;Qy), the grid of equation (stretch) over the full channel (or over the
right half, with the point symmetry of Sec. II at x = 0, when ``half_channel`` is set), the
rarefaction parameter delta of equation (delta), wall speed, wall temperature, Prandtl number
and the viscosity index of equation (mu).  Every array is float64, velocities ordered
v = (h*Qx + i)*Qy + j (h = 0: p_x = +z_i, h = 1: p_x = -z_i), cells contiguous.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading

import numpy as np

from . import quadrature as quad

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hrlb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_hrlb.so")
_lock = threading.Lock()
_lib = None

FIELD_NAMES = ("n", "u_x", "u_y", "T", "P_xx", "P_xy", "P_yy", "T_zz", "q_x", "q_y")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC,
               "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("Qx", C.c_int), ("Nx", C.c_int), ("Qy", C.c_int), ("Ny", C.c_int),
        ("zx", C.POINTER(C.c_double)), ("wx", C.POINTER(C.c_double)),
        ("phi_hi", C.POINTER(C.c_double)), ("phi_lo", C.POINTER(C.c_double)),
        ("zy", C.POINTER(C.c_double)), ("wy", C.POINTER(C.c_double)),
        ("ncell", C.c_int), ("stretch_A", C.c_double),
        ("delta", C.c_double), ("uw", C.c_double), ("Tw", C.c_double), ("Pr", C.c_double),
        ("omega", C.c_double), ("dt", C.c_double), ("collisionless", C.c_int), ("half", C.c_int),
        ("ntab", C.c_int), ("tabT", C.POINTER(C.c_double)), ("tabMu", C.POINTER(C.c_double)),
        ("tabPr", C.POINTER(C.c_double)), ("lts_cap", C.c_double), ("wall_closure", C.c_int),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = C.CDLL(build())
            dp = C.POINTER(C.c_double)
            pp = C.POINTER(_Problem)
            lib.orc_grid.argtypes = [pp, dp, dp, dp]
            lib.orc_gx.argtypes = [pp, C.c_double, C.c_double, dp]
            lib.orc_gy.argtypes = [pp, C.c_double, C.c_double, dp]
            lib.orc_moments.argtypes = [pp, dp, dp, dp]
            lib.orc_tau.argtypes = [pp, C.c_double, C.c_double]
            lib.orc_tau.restype = C.c_double
            lib.orc_prandtl.argtypes = [pp, C.c_double]
            lib.orc_prandtl.restype = C.c_double
            lib.orc_collision_target.argtypes = [pp, dp, dp, dp]
            lib.orc_weno5.argtypes = [C.c_double] * 5
            lib.orc_weno5.restype = C.c_double
            lib.orc_weno5_sub.argtypes = [C.c_double] * 5 + [C.c_int]
            lib.orc_weno5_sub.restype = C.c_double
            lib.orc_row_faces.argtypes = [pp, C.c_double, dp, C.c_double, C.c_double, dp, dp, dp]
            lib.orc_rhs.argtypes = [pp, dp, dp, dp, dp, dp]
            lib.orc_init_state.argtypes = [pp, dp, dp]
            lib.orc_step.argtypes = [pp, dp, dp, C.c_long, C.c_int, C.c_double, dp]
            lib.orc_step.restype = C.c_long
            lib.orc_num_threads.restype = C.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def weno5(a, b, c, d, e) -> float:
    """WENO-5 face value from five values ordered along the upwind direction (c = upwind cell)."""
    return _load().orc_weno5(a, b, c, d, e)


def weno5_sub(a, b, c, d, e, mask: int) -> float:
    """WENO-5 with only the candidate stencils of mask (bit k: stencil k) and renormalised linear weights."""
    return _load().orc_weno5_sub(a, b, c, d, e, mask)


def num_threads() -> int:
    return _load().orc_num_threads()


class OracleProblem:
    """One Couette case for the FP64 oracle."""

    def __init__(self, Qx: int, Qy: int, ncell: int, *, Nx: int | None = None, Ny: int | None = None,
                 stretch_A: float = 0.0, delta: float = 1.0, uw: float = 0.05, Tw: float = 1.0,
                 Pr: float = 2.0 / 3.0, omega: float = 0.7, dt: float | None = None, cfl: float = 0.5,
                 collisionless: bool = False, half_channel: bool = False, visc_table=None,
                 local_dt_cap: float = 0.0, wall_closure: int = 0):
        self.Qx, self.Qy = Qx, Qy
        self.Nx = min(Qx - 1, 10) if Nx is None else Nx
        self.Ny = Qy - 1 if Ny is None else Ny
        self.ncell, self.stretch_A = ncell, stretch_A
        self.half = bool(half_channel)
        # equations (mun), (interp): rows (T_n, mu_n, Pr_n) with T_n ascending; replaces omega and Pr
        self.table = None if visc_table is None else np.ascontiguousarray(np.asarray(visc_table, np.float64).T)
        self.delta, self.uw, self.Tw, self.Pr, self.omega = delta, uw, Tw, Pr, omega
        self.collisionless = bool(collisionless or delta == 0.0)
        hr = quad.half_range_rule(Qx)
        fr = quad.full_range_rule(Qy)
        self.zx, self.wx = hr.nodes_f64(), hr.weights_f64()
        self.zy, self.wy = fr.nodes_f64(), fr.weights_f64()
        phi = quad.phi_table(Qx, self.Nx)
        hi, lo = quad.split_hi_lo([v for row in phi for v in row])
        self.phi_hi, self.phi_lo = hi, lo
        self.nv = 2 * Qx * Qy
        px = np.concatenate([self.zx, -self.zx])
        self.px = np.repeat(px, Qy)
        self.py = np.tile(self.zy, 2 * Qx)
        self._keep = [self.zx, self.wx, self.zy, self.wy, self.phi_hi, self.phi_lo]
        if self.table is not None:
            assert self.table.shape[0] == 3 and self.table.shape[1] >= 2
            self._tab = [np.ascontiguousarray(r) for r in self.table]
            self._keep += self._tab
        self.x, self.J, self.deta = self._grid()
        if dt is None:
            dt = self.default_dt(cfl)
        self.dt = float(dt)
        self._p = _Problem(Qx, self.Nx, Qy, self.Ny, _ptr(self.zx), _ptr(self.wx), _ptr(self.phi_hi),
                           _ptr(self.phi_lo), _ptr(self.zy), _ptr(self.wy), ncell, stretch_A,
                           delta, uw, Tw, Pr, omega, self.dt, int(self.collisionless), int(self.half),
                           0 if self.table is None else self.table.shape[1],
                           *([None] * 3 if self.table is None else [_ptr(r) for r in self._tab]),
                           float(local_dt_cap), int(wall_closure))

    # -- grid and time step ------------------------------------------------------------------
    def _grid(self):
        N = self.ncell
        if self.half:
            # equation (stretch) as the paper states it: eta_s = (s - 1/2) artanh(A)/S, s = 1..S
            if self.stretch_A == 0.0:
                deta = 0.5 / N
                return (np.arange(N) + 0.5) * deta, np.ones(N), deta
            A = self.stretch_A
            deta = math.atanh(A) / N
            eta = (np.arange(N) + 0.5) * deta
            return np.tanh(eta) / (2 * A), 1.0 / (2 * A * np.cosh(eta) ** 2), deta
        if self.stretch_A == 0.0:
            deta = 1.0 / N
            x = -0.5 + (np.arange(N) + 0.5) / N
            J = np.ones(N)
        else:
            A = self.stretch_A
            emax = math.atanh(A)
            deta = 2 * emax / N
            eta = -emax + (np.arange(N) + 0.5) * deta
            x = np.tanh(eta) / (2 * A)
            J = 1.0 / (2 * A * np.cosh(eta) ** 2)
        return x, J, deta

    def default_dt(self, cfl: float = 0.5) -> float:
        """dt = min(CFL min_s(J_s deta)/max|p_x|, tau(n=1, T_w)/2); tau is dropped when collisionless."""
        adv = cfl * float(np.min(self.J)) * self.deta / float(np.max(self.zx))
        if self.collisionless:
            return adv
        tau_w = 1.0 / (self.delta * math.sqrt(2.0)) / math.sqrt(self.Tw)
        return min(adv, 0.5 * tau_w)

    # -- pieces --------------------------------------------------------------------------------
    def gx(self, u: float, T: float) -> np.ndarray:
        out = np.zeros(2 * self.Qx)
        if _load().orc_gx(C.byref(self._p), u, T, _ptr(out)) != 0:
            raise ValueError("orc_gx failed")
        return out

    def gy(self, u: float, T: float) -> np.ndarray:
        out = np.zeros(self.Qy)
        if _load().orc_gy(C.byref(self._p), u, T, _ptr(out)) != 0:
            raise ValueError("orc_gy failed")
        return out

    def tau(self, n: float, T: float) -> float:
        return _load().orc_tau(C.byref(self._p), n, T)

    def prandtl(self, T: float) -> float:
        return _load().orc_prandtl(C.byref(self._p), T)

    def collision_target(self, n, ux, uy, T, qx, qy):
        cell = np.array([n, ux, uy, T, qx, qy], dtype=np.float64)
        tp, tc = np.zeros(self.nv), np.zeros(self.nv)
        _load().orc_collision_target(C.byref(self._p), _ptr(cell), _ptr(tp), _ptr(tc))
        return tp, tc

    def row_faces(self, px: float, f: np.ndarray, wall_l: float = 0.0, wall_r: float = 0.0, fm=None):
        """(extended row over cells -3 .. N+2, the N+1 face values) of one velocity's row f as the
        right-hand side builds them: ghosts, wall populations wall_l / wall_r of entering directions,
        the mirrored row fm of the half channel."""
        f = np.ascontiguousarray(f, np.float64)
        e, F = np.zeros(self.ncell + 6), np.zeros(self.ncell + 1)
        fmp = None if fm is None else _ptr(np.ascontiguousarray(fm, np.float64))
        if _load().orc_row_faces(C.byref(self._p), px, _ptr(f), wall_l, wall_r, fmp, _ptr(e), _ptr(F)) != 0:
            raise ValueError("orc_row_faces failed")
        return e, F

    def init_state(self):
        phi = np.zeros((self.nv, self.ncell))
        chi = np.zeros((self.nv, self.ncell))
        _load().orc_init_state(C.byref(self._p), _ptr(phi), _ptr(chi))
        return phi, chi

    def moments(self, phi: np.ndarray, chi: np.ndarray) -> np.ndarray:
        phi, chi = np.ascontiguousarray(phi, np.float64), np.ascontiguousarray(chi, np.float64)
        out = np.zeros((10, self.ncell))
        _load().orc_moments(C.byref(self._p), _ptr(phi), _ptr(chi), _ptr(out))
        return out

    def rhs(self, phi: np.ndarray, chi: np.ndarray):
        phi, chi = np.ascontiguousarray(phi, np.float64), np.ascontiguousarray(chi, np.float64)
        dp, dc = np.zeros_like(phi), np.zeros_like(chi)
        info = np.zeros(4)
        if _load().orc_rhs(C.byref(self._p), _ptr(phi), _ptr(chi), _ptr(dp), _ptr(dc), _ptr(info)) != 0:
            raise ValueError("orc_rhs failed")
        return dp, dc, info

    def step(self, phi: np.ndarray, chi: np.ndarray, n_steps: int, check_every: int = 0,
             tol: float = 0.0):
        """Advance in place; returns (steps_taken, last_residual)."""
        assert phi.flags.c_contiguous and chi.flags.c_contiguous
        res = C.c_double(-1.0)
        taken = _load().orc_step(C.byref(self._p), _ptr(phi), _ptr(chi), n_steps, check_every, tol,
                                 C.byref(res))
        if taken < 0:
            raise MemoryError("orc_step failed")
        return int(taken), res.value

    # -- outputs -------------------------------------------------------------------------------
    def mass(self, phi: np.ndarray) -> float:
        return float(np.sum(self.J * self.deta * phi.sum(axis=0)))

    def mean_pxy(self, fields: np.ndarray) -> float:
        w = self.J * self.deta
        return float(np.sum(w * fields[5]) / np.sum(w))

    def Pi(self, fields: np.ndarray) -> float:
        """Equation (Pi): Pi = -T_xy v_ref/(P_ref u_w sqrt 2), T_xy the J-weighted channel mean."""
        vref, pref = math.sqrt(self.Tw), self.Tw
        return -self.mean_pxy(fields) * vref / (pref * self.uw * math.sqrt(2.0))

"""Thin Python binding of libhrlb (include/hrlb.h) through ctypes.

Argument marshalling only: every step of the solver runs in the HIP kernels of libhrlb.so.
PyTorch supplies the device workspace (a uint8 tensor) and the HIP stream.  If the library is
missing, loading fails loudly; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhrlb.so")

HRLB_OK, HRLB_NOT_CONVERGED = 0, 1
HRLB_E_INVALID, HRLB_E_NOMEM, HRLB_E_DEVICE, HRLB_E_DIVERGED, HRLB_E_RANGE = -1, -2, -3, -4, -5
HRLB_FLAG_NONFINITE, HRLB_FLAG_RANGE = 1, 2
HRLB_FP64, HRLB_FP32_STORE_FP64_MOM = 0, 1
HRLB_ROUND_NEAREST, HRLB_ROUND_STOCHASTIC = 0, 1
HRLB_STOP_RESIDUAL, HRLB_STOP_PXY, HRLB_STOP_PXY_ERR = 0, 1, 2
HRLB_PATH_AUTO, HRLB_PATH_TILED, HRLB_PATH_SMALL = 0, 1, 2

FIELD_NAMES = ("n", "u_x", "u_y", "T", "P_xx", "P_xy", "P_yy", "T_zz", "q_x", "q_y")

EXPORTED = (
    "hrlb_init_quadrature", "hrlb_quadrature_nodes", "hrlb_case_workspace_bytes", "hrlb_init_case",
    "hrlb_case_state_bytes", "hrlb_init_case_static",
    "hrlb_step", "hrlb_run_to_steady", "hrlb_moments", "hrlb_get_state", "hrlb_set_state",
    "hrlb_case_info", "hrlb_case_flags", "hrlb_case_kernel_path", "hrlb_free_case", "hrlb_free_quadrature", "hrlb_last_error",
    "hrlb_batch_workspace_bytes", "hrlb_batch_create", "hrlb_batch_step", "hrlb_batch_poll",
    "hrlb_batch_free", "hrlb_batch_profile", "hrlb_batch_set_streams", "hrlb_case_set_graph_steps",
    "hrlb_batch_set_graph_steps",
    "hrlb_tune_workspace_bytes", "hrlb_tune_plan",
    "hrlb_server_create", "hrlb_server_clock", "hrlb_server_submit", "hrlb_server_pump", "hrlb_server_request",
    "hrlb_server_free", "hrlb_average_start", "hrlb_average_stop", "hrlb_average_read",
    "hrlb_pxy_error_estimate",
)
HRLB_REQ_WAITING, HRLB_REQ_ACTIVE, HRLB_REQ_DONE, HRLB_REQ_FAILED = 0, 1, 2, 3


class HrlbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hrlb status {status}: {msg}")
        self.status = status


class CaseParams(C.Structure):
    _fields_ = [
        ("delta", C.c_double), ("u_w", C.c_double), ("T_w", C.c_double), ("Pr", C.c_double),
        ("omega", C.c_double), ("n_cells", C.c_int), ("stretch_A", C.c_double),
        ("precision", C.c_int), ("rounding", C.c_int), ("cfl", C.c_double), ("dt", C.c_double),
        ("seed", C.c_uint), ("tile_vpt", C.c_int), ("cell_lanes", C.c_int), ("half_channel", C.c_int),
        ("visc_table_n", C.c_int), ("visc_T", C.POINTER(C.c_double)), ("visc_mu", C.POINTER(C.c_double)),
        ("visc_Pr", C.POINTER(C.c_double)), ("local_dt_cap", C.c_double), ("kernel_path", C.c_int),
    ]


class SteadyInfo(C.Structure):
    _fields_ = [("steps", C.c_long), ("residual", C.c_double), ("pxy_drift", C.c_double),
                ("sim_time", C.c_double), ("wall_s", C.c_double), ("mass_drift", C.c_double),
                ("pxy_err", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("max_active", C.c_int), ("check_every", C.c_int), ("max_bypass", C.c_int), ("precision", C.c_int)]


class SolveRequest(C.Structure):
    _fields_ = [("Qx", C.c_int), ("Nx_order", C.c_int), ("Qy", C.c_int), ("Ny_order", C.c_int),
                ("params", CaseParams), ("tol", C.c_double), ("stop_rule", C.c_int), ("max_steps", C.c_long),
                ("arrival_s", C.c_double)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int), ("status", C.c_int), ("steps", C.c_long), ("residual", C.c_double),
                ("pxy_drift", C.c_double), ("Pi", C.c_double), ("sim_time", C.c_double),
                ("mass_drift", C.c_double), ("pxy_err", C.c_double), ("t_arrival", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("n_cells", C.c_int), ("n_vel", C.c_int), ("bytes", C.c_size_t)]


class ServerStats(C.Structure):
    _fields_ = [("waiting", C.c_int), ("active", C.c_int), ("done", C.c_int), ("failed", C.c_int),
                ("admitted", C.c_int), ("retired", C.c_int), ("steps", C.c_long), ("units", C.c_double),
                ("round_s", C.c_double), ("arena_used", C.c_size_t), ("arena_largest_free", C.c_size_t)]


_lib = None
_lock = threading.Lock()


def load() -> C.CDLL:
    """Load libhrlb.so (built by paper_1810_07803_amd/build.py); raise if it is absent."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1810_07803_amd.build")
            # torch ships its own HIP runtime (same soname); loading it first makes libhrlb bind to
            # that runtime, so torch's device pointers and streams are valid inside the library
            import torch  # noqa: F401

            lib = C.CDLL(LIB_PATH)
            vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
            sig = {
                "hrlb_init_quadrature": [C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.POINTER(vp)],
                "hrlb_quadrature_nodes": [vp, dp, dp, dp, dp],
                "hrlb_case_workspace_bytes": [vp, C.POINTER(CaseParams), C.POINTER(C.c_size_t)],
                "hrlb_init_case": [vp, C.POINTER(CaseParams), vp, C.c_size_t, vp, C.POINTER(vp)],
                "hrlb_case_state_bytes": [vp, C.POINTER(CaseParams), C.POINTER(C.c_size_t)],
                "hrlb_init_case_static": [vp, C.POINTER(CaseParams), vp, C.c_size_t, vp, C.POINTER(vp)],
                "hrlb_step": [vp, C.c_long],
                "hrlb_run_to_steady": [vp, C.c_double, C.c_long, C.c_int, C.c_int, C.POINTER(SteadyInfo)],
                "hrlb_moments": [vp, dp, dp, dp, dp],
                "hrlb_get_state": [vp, dp],
                "hrlb_set_state": [vp, dp],
                "hrlb_case_info": [vp, dp, ip, ip, C.POINTER(C.c_long)],
                "hrlb_case_flags": [vp, C.POINTER(C.c_uint)],
                "hrlb_case_kernel_path": [vp, ip],
                "hrlb_batch_workspace_bytes": [C.POINTER(vp), C.c_int, C.POINTER(C.c_size_t)],
                "hrlb_batch_create": [C.POINTER(vp), C.c_int, vp, C.c_size_t, C.POINTER(vp)],
                "hrlb_batch_step": [vp, C.c_long, C.c_int],
                "hrlb_batch_poll": [vp, dp, dp],
                "hrlb_batch_profile": [vp, C.c_long, dp, dp],
                "hrlb_case_set_graph_steps": [vp, C.c_int],
                "hrlb_tune_workspace_bytes": [vp, C.POINTER(CaseParams), C.POINTER(C.c_size_t)],
                "hrlb_tune_plan": [vp, C.POINTER(CaseParams), vp, C.c_size_t, vp, C.c_int, ip, ip, dp],
                "hrlb_batch_set_graph_steps": [vp, C.c_int],
                "hrlb_batch_set_streams": [vp, C.c_int],
                "hrlb_average_start": [vp],
                "hrlb_average_stop": [vp],
                "hrlb_average_read": [vp, dp, dp, C.POINTER(C.c_long)],
                "hrlb_server_create": [C.POINTER(ServerConfig), vp, C.c_size_t, vp, C.POINTER(vp)],
                "hrlb_server_submit": [vp, C.POINTER(SolveRequest), C.POINTER(C.c_long)],
                "hrlb_server_pump": [vp, C.POINTER(ServerStats)],
                "hrlb_server_request": [vp, C.c_long, C.POINTER(RequestInfo), dp, dp, C.c_int],
                "hrlb_pxy_error_estimate": [dp, C.c_int, dp],
            }
            for name, args in sig.items():
                fn = getattr(lib, name)
                fn.argtypes = args
                fn.restype = C.c_int
            lib.hrlb_server_clock.argtypes = [vp]
            lib.hrlb_server_clock.restype = C.c_double
            for name in ("hrlb_free_case", "hrlb_free_quadrature", "hrlb_batch_free", "hrlb_server_free"):
                getattr(lib, name).argtypes = [vp]
                getattr(lib, name).restype = None
            lib.hrlb_last_error.argtypes = []
            lib.hrlb_last_error.restype = C.c_char_p
            _lib = lib
    return _lib


def pxy_error_estimate(means) -> float:
    """The estimate behind HRLB_STOP_PXY_ERR for successive checked means of P_xy (host only)."""
    m = np.ascontiguousarray(means, dtype=np.float64)
    est = C.c_double()
    _check(load().hrlb_pxy_error_estimate(_dptr(m), len(m), C.byref(est)))
    return est.value


def _check(status: int, allow=(HRLB_OK,)) -> int:
    if status not in allow:
        raise HrlbError(status, load().hrlb_last_error().decode(errors="replace"))
    return status


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---- velocity set ------------------------------------------------------------------------------
class Quadrature:
    """HHLB(Nx;Qx) x HLB(Ny;Qy) velocity set (hrlb_init_quadrature)."""

    def __init__(self, Qx: int, Qy: int, Nx: int | None = None, Ny: int | None = None, p0: float = 1.0):
        self.Qx, self.Qy = Qx, Qy
        self.Nx = min(Qx - 1, 10) if Nx is None else Nx
        self.Ny = Qy - 1 if Ny is None else Ny
        h = C.c_void_p()
        _check(load().hrlb_init_quadrature(Qx, self.Nx, Qy, self.Ny, p0, C.byref(h)))
        self.handle = h

    def nodes(self):
        px, wx = np.zeros(2 * self.Qx), np.zeros(2 * self.Qx)
        py, wy = np.zeros(self.Qy), np.zeros(self.Qy)
        _check(load().hrlb_quadrature_nodes(self.handle, _dptr(px), _dptr(wx), _dptr(py), _dptr(wy)))
        return px, wx, py, wy

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hrlb_free_quadrature(self.handle)
            self.handle = None


def init_quadrature(Qx, Nx, Qy, Ny, p0=1.0) -> Quadrature:
    return Quadrature(Qx, Qy, Nx, Ny, p0)


def make_params(*, delta, uw, ncell, stretch_A=0.0, Tw=1.0, Pr=2.0 / 3.0, omega=0.7, precision=HRLB_FP64,
                rounding=HRLB_ROUND_NEAREST, cfl=0.5, dt=0.0, seed=0, tile_vpt=0, cell_lanes=0,
                half_channel=0, visc_table=None, local_dt_cap=0.0, kernel_path=HRLB_PATH_AUTO) -> CaseParams:
    """Case parameters.  visc_table: rows (T_k, mu_k, Pr_k) of the tabulated transport law (copied by
    the library when the case is created; the returned struct keeps the arrays alive until then)."""
    p = CaseParams(delta, uw, Tw, Pr, omega, ncell, stretch_A, precision, rounding, cfl, dt, seed & 0xFFFFFFFF,
                   tile_vpt, cell_lanes, int(half_channel))
    p.local_dt_cap = float(local_dt_cap)
    p.kernel_path = int(kernel_path)
    if visc_table is not None:
        cols = [np.ascontiguousarray(c, dtype=np.float64) for c in np.asarray(visc_table, np.float64).T]
        p.visc_table_n = len(cols[0])
        p.visc_T, p.visc_mu, p.visc_Pr = (_dptr(c) for c in cols)
        p._visc_keep = cols
    return p


def tune_plan(quad: "Quadrature", params: CaseParams, n_steps: int = 20, device="cuda:0"):
    """Autotune the kernel plan of one case (hrlb_tune_plan): returns (tile_vpt, cell_lanes, ms_per_step)."""
    import torch

    n = C.c_size_t()
    _check(load().hrlb_tune_workspace_bytes(quad.handle, C.byref(params), C.byref(n)))
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
    base = ws.data_ptr()
    off = (-base) % 256
    stream = torch.cuda.current_stream(device)
    bv, bl, ms = C.c_int(), C.c_int(), C.c_double()
    _check(load().hrlb_tune_plan(quad.handle, C.byref(params), C.c_void_p(base + off), n.value,
                                 C.c_void_p(stream.cuda_stream), n_steps, C.byref(bv), C.byref(bl), C.byref(ms)))
    return bv.value, bl.value, ms.value


def workspace_bytes(quad: Quadrature, params: CaseParams) -> int:
    n = C.c_size_t()
    _check(load().hrlb_case_workspace_bytes(quad.handle, C.byref(params), C.byref(n)))
    return n.value


# ---- one case ----------------------------------------------------------------------------------
def state_bytes(quad: Quadrature, params: CaseParams) -> int:
    n = C.c_size_t()
    _check(load().hrlb_case_state_bytes(quad.handle, C.byref(params), C.byref(n)))
    return n.value


class Case:
    """One Couette problem resident in a torch-allocated device workspace (hrlb_init_case).  With
    static=True the caller's memory holds the populations only and the rest of the case lives in the
    library's static scratch (hrlb_init_case_static; one such case per device at a time)."""

    def __init__(self, quad: Quadrature, params: CaseParams, device="cuda:0", stream=None, workspace=None,
                 static: bool = False):
        import torch

        self.quad, self.params = quad, params
        nbytes = state_bytes(quad, params) if static else workspace_bytes(quad, params)
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._ws_tensor = workspace
        base = workspace.data_ptr()
        off = (-base) % 256
        if workspace.numel() - off < nbytes:
            raise HrlbError(HRLB_E_NOMEM, "workspace tensor too small")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        init = load().hrlb_init_case_static if static else load().hrlb_init_case
        _check(init(quad.handle, C.byref(params), C.c_void_p(base + off), nbytes,
                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        dt, nv, nc, sd = C.c_double(), C.c_int(), C.c_int(), C.c_long()
        _check(load().hrlb_case_info(h, C.byref(dt), C.byref(nv), C.byref(nc), C.byref(sd)))
        self.dt, self.nv, self.ncell = dt.value, nv.value, nc.value
        self.workspace_bytes = nbytes

    def step(self, n_steps: int):
        _check(load().hrlb_step(self.handle, n_steps))

    def run_to_steady(self, tol: float, max_steps: int, check_every: int = 100, stop_rule: int = HRLB_STOP_RESIDUAL):
        info = SteadyInfo()
        st = _check(load().hrlb_run_to_steady(self.handle, tol, max_steps, check_every, stop_rule, C.byref(info)),
                    allow=(HRLB_OK, HRLB_NOT_CONVERGED))
        return st, info

    def moments(self):
        f = np.zeros((10, self.ncell))
        x = np.zeros(self.ncell)
        pi = C.c_double()
        sh = np.zeros(2)
        _check(load().hrlb_moments(self.handle, _dptr(f), _dptr(x), C.byref(pi), _dptr(sh)))
        return f, x, pi.value, sh

    def get_state(self) -> np.ndarray:
        s = np.zeros((2, self.nv, self.ncell))
        _check(load().hrlb_get_state(self.handle, _dptr(s)))
        return s

    def set_state(self, state: np.ndarray):
        s = np.ascontiguousarray(state, dtype=np.float64)
        assert s.shape == (2, self.nv, self.ncell)
        _check(load().hrlb_set_state(self.handle, _dptr(s)))

    def set_graph_steps(self, steps: int):
        """Steps per captured HIP graph (0 disables graphs)."""
        _check(load().hrlb_case_set_graph_steps(self.handle, steps))

    def average_start(self):
        """Start time-averaging the fields over the steps completed from now on."""
        _check(load().hrlb_average_start(self.handle))

    def average_stop(self):
        _check(load().hrlb_average_stop(self.handle))

    def average_read(self):
        """(fields [10][n_cells], Pi, steps) averaged since average_start."""
        f = np.zeros((10, self.ncell))
        pi, n = C.c_double(), C.c_long()
        _check(load().hrlb_average_read(self.handle, _dptr(f), C.byref(pi), C.byref(n)))
        return f, pi.value, n.value

    def flags(self) -> int:
        """Sticky condition bits (HRLB_FLAG_NONFINITE, HRLB_FLAG_RANGE)."""
        f = C.c_uint()
        _check(load().hrlb_case_flags(self.handle, C.byref(f)))
        return f.value

    def kernel_path(self) -> int:
        """HRLB_PATH_TILED or HRLB_PATH_SMALL: the kernels that advance this case."""
        p = C.c_int()
        _check(load().hrlb_case_kernel_path(self.handle, C.byref(p)))
        return p.value

    def steps_done(self) -> int:
        sd = C.c_long()
        _check(load().hrlb_case_info(self.handle, None, None, None, C.byref(sd)))
        return sd.value

    def free(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hrlb_free_case(self.handle)
            self.handle = None

    def __del__(self):
        self.free()


def init_case(quad, params, device="cuda:0", stream=None) -> Case:
    return Case(quad, params, device, stream)


# ---- batches -----------------------------------------------------------------------------------
class Batch:
    """Several cases advanced by shared launches (hrlb_batch_create)."""

    def __init__(self, cases, device="cuda:0"):
        import torch

        self.cases = list(cases)
        arr = (C.c_void_p * len(self.cases))(*[c.handle.value for c in self.cases])
        n = C.c_size_t()
        _check(load().hrlb_batch_workspace_bytes(arr, len(self.cases), C.byref(n)))
        self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        _check(load().hrlb_batch_create(arr, len(self.cases), C.c_void_p(base + off), n.value, C.byref(h)))
        self.handle = h

    def step(self, n_steps: int, check: bool = False):
        _check(load().hrlb_batch_step(self.handle, n_steps, int(check)))

    def poll(self):
        r = np.zeros(len(self.cases))
        p = np.zeros(len(self.cases))
        _check(load().hrlb_batch_poll(self.handle, _dptr(r), _dptr(p)))
        return r, p

    def set_graph_steps(self, steps: int):
        """Steps per captured HIP graph (0 disables graphs)."""
        _check(load().hrlb_batch_set_graph_steps(self.handle, steps))

    def set_streams(self, n: int):
        """Advance the batch as n parts of about equal work, each on its own stream (1..4)."""
        _check(load().hrlb_batch_set_streams(self.handle, n))

    def profile(self, n_steps: int):
        """Mean duration (ms) of one stage-kernel launch and one per-cell-kernel launch."""
        a, b = C.c_double(), C.c_double()
        _check(load().hrlb_batch_profile(self.handle, n_steps, C.byref(a), C.byref(b)))
        return a.value, b.value

    def free(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hrlb_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        self.free()


# ---- serving -----------------------------------------------------------------------------------
class Server:
    """Request loop with continuous batching over one torch-allocated device arena (hrlb_server_*)."""

    def __init__(self, arena_bytes: int, *, max_active: int = 64, check_every: int = 200, max_bypass: int = 4,
                 precision: int = HRLB_FP32_STORE_FP64_MOM, device="cuda:0", stream=None):
        import torch

        self.check_every, self.precision = check_every, precision
        self._arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=device)
        base = self._arena.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        cfg = ServerConfig(max_active, check_every, max_bypass, precision)
        h = C.c_void_p()
        _check(load().hrlb_server_create(C.byref(cfg), C.c_void_p(base + off), arena_bytes,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h
        self._ncell = {}

    def clock(self) -> float:
        return load().hrlb_server_clock(self.handle)

    def submit(self, Qx: int, Qy: int, params: CaseParams, *, tol: float, max_steps: int,
               stop_rule: int = HRLB_STOP_PXY, Nx: int | None = None, Ny: int | None = None,
               arrival_s: float = -1.0) -> int:
        nxo = min(Qx - 1, 10) if Nx is None else Nx
        nyo = Qy - 1 if Ny is None else Ny
        req = SolveRequest(Qx, nxo, Qy, nyo, params, tol, stop_rule, max_steps, arrival_s)
        rid = C.c_long()
        _check(load().hrlb_server_submit(self.handle, C.byref(req), C.byref(rid)))
        self._ncell[rid.value] = params.n_cells
        return rid.value

    def pump(self) -> ServerStats:
        st = ServerStats()
        _check(load().hrlb_server_pump(self.handle, C.byref(st)))
        return st

    def request(self, rid: int, release: bool = False):
        """(info, fields [10][n_cells] or None, x or None) of a request."""
        info = RequestInfo()
        if rid not in self._ncell:  # unknown or released: the library reports the error
            _check(load().hrlb_server_request(self.handle, rid, C.byref(info), None, None, 0))
        n = self._ncell[rid]
        f, x = np.zeros((10, n)), np.zeros(n)
        _check(load().hrlb_server_request(self.handle, rid, C.byref(info), _dptr(f), _dptr(x), int(release)))
        if release and info.state in (HRLB_REQ_DONE, HRLB_REQ_FAILED):
            self._ncell.pop(rid, None)
        if info.state != HRLB_REQ_DONE:
            return info, None, None
        return info, f, x

    def free(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hrlb_server_free(self.handle)
            self.handle = None

    def __del__(self):
        self.free()

"""Edge sizes of the C ABI against the oracle: the smallest grid (8 cells, both walls' stencils
overlapping) with the smallest velocity set, the largest velocity set (Qx = 128, Qy = 64: 16384
velocities, the runtime-order g_y path), and the highest expansion order of eq. (gx) (N_x = 16)."""
import numpy as np
import pytest

from hrlb_inputs import perturb
from tests.gpu_helpers import make_pair, parity, say

pytestmark = pytest.mark.gpu


def _parity(Qx, Qy, nx, steps, tol, *, precision=0, rounding=0, Nx=None, half=False, tile_vpt=0, path=1, **kw):
    from oracle.oracle import OracleProblem
    from paper_1810_07803_amd import hrlb

    orc = OracleProblem(Qx, Qy, nx, Nx=Nx, half_channel=half, **kw)
    q = hrlb.Quadrature(Qx, Qy, orc.Nx, orc.Ny)
    case = hrlb.Case(q, hrlb.make_params(delta=kw["delta"], uw=kw["uw"], ncell=nx, stretch_A=kw.get("stretch_A", 0.0),
                                         precision=precision, rounding=rounding, dt=orc.dt, seed=5,
                                         half_channel=int(half), tile_vpt=tile_vpt, kernel_path=path))
    case._quad_ref = q
    phi, chi = orc.init_state()
    phi, chi = perturb(phi, 0.05, 61), perturb(chi, 0.05, 62)
    case.set_state(np.stack([phi, chi]))
    case.step(steps)
    orc.step(phi, chi, steps)
    say(f"   Q{Qx}x{Qy} Nx={orc.Nx} Ny={orc.Ny} nx={nx} half={half} precision={precision}")
    return parity(case.get_state(), phi, chi, case.moments()[0], orc.moments(phi, chi), tol)


@pytest.mark.parametrize("precision,rounding,tol", [(0, 0, 1e-12), (1, 1, 1e-5)])
@pytest.mark.parametrize("half", [False, True])
@pytest.mark.parametrize("path", [1, 2])
def test_smallest_grid_and_velocity_set(precision, rounding, tol, half, path):
    say(f"[extremes] 8 cells, HHLB(2;3) x HLB(2;3), kernel path {path}")
    assert _parity(3, 3, 8, 30, tol, precision=precision, rounding=rounding, half=half, delta=1.0, uw=0.4,
                   stretch_A=0.9, path=path)


@pytest.mark.parametrize("precision,rounding,tol", [(0, 0, 1e-12), (1, 1, 1e-5)])
def test_largest_velocity_set(precision, rounding, tol):
    # FP32 storage: the stage kernel's LDS (cell tables of 64 g_y rows, the per-tile velocity
    # tables, the window prefetch buffers) is at its largest here
    say("[extremes] HHLB(10;128) x HLB(63;64): 16384 velocities, 8 cells")
    assert _parity(128, 64, 8, 3, tol, precision=precision, rounding=rounding, delta=1.0, uw=0.3, stretch_A=0.9)


@pytest.mark.parametrize("half", [False, True])
def test_longest_rows_fp32(half):
    # rows of 16 velocities (the most a row holds): the prefetch walks 16 velocities per tile and the
    # per-tile copies of p_y and the wall populations are at their largest; 96 cells = one full tile
    # and a ragged one
    say(f"[extremes] rows of 16 velocities, HHLB(7;8) x HLB(15;16), 96 cells, half={half}")
    assert _parity(8, 16, 96, 12, 1e-5, precision=1, rounding=1, half=half, tile_vpt=16, delta=0.5, uw=0.3,
                   stretch_A=0.9)


def test_highest_expansion_order_of_gx():
    say("[extremes] HHLB(16;32) x HLB(7;8), 40 cells")
    assert _parity(32, 8, 40, 10, 1e-12, Nx=16, delta=0.5, uw=0.3, stretch_A=0.9)


def test_zero_steps_leave_the_state_unchanged():
    # n_steps = 0 on a case and on a batch, and a checked zero-step batch call, do nothing
    from paper_1810_07803_amd import hrlb

    say("[extremes] zero-step calls")
    case, _ = make_pair(8, 4, 64, delta=1.0, uw=0.3, stretch_A=0.9)
    case.step(3)
    s0 = case.get_state()
    f0 = case.moments()[0]
    case.step(0)
    b = hrlb.Batch([case])
    b.step(0)
    b.step(0, check=True)
    np.testing.assert_array_equal(case.get_state(), s0)
    np.testing.assert_array_equal(case.moments()[0], f0)
    assert case.steps_done() == 3

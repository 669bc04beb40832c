"""CPU regression test of the stage kernel's work lists: a case's or batch's tile list must match
its allocated length record for record (a mismatch once made the kernel read stale records)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tile_lists_cover_every_tile_once_and_fit_their_capacity(tmp_path):
    exe = tmp_path / "plan_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_1810_07803_amd", "csrc"),
                    os.path.join(ROOT, "tests", "plan_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr


def test_workspace_query_validates_the_case_tile_list():
    from paper_1810_07803_amd import hrlb

    for qx, qy in ((4, 4), (8, 12), (16, 7), (32, 8), (80, 20)):
        q = hrlb.Quadrature(qx, qy)
        for ncell in (8, 12, 64, 68, 100, 1024, 2048):
            for vpt in (0, 1):
                assert hrlb.workspace_bytes(q, hrlb.make_params(delta=1.0, uw=0.1, ncell=ncell, tile_vpt=vpt)) > 0


def test_long_row_plan_of_the_batch_workloads():
    # the rows the benchmark's batches ask for: the largest divisor of Q_y up to 16 that leaves at
    # least 16 rows (2 Q_x Q_y / vpt >= 16), checked against brute force over all admissible plans
    import bench

    for Qx in (3, 4, 8, 16, 32, 80, 128):
        for Qy in (3, 4, 6, 8, 12, 16, 20, 64):
            v = bench.long_row_vpt(Qx, Qy)
            ok = [d for d in range(1, 17) if Qy % d == 0 and 2 * Qx * Qy // d >= 16]
            assert v == max(ok), (Qx, Qy, v)
    assert bench.long_row_vpt(8, 12) == 12 and bench.long_row_vpt(4, 12) == 6 and bench.long_row_vpt(4, 4) == 2

"""Writes tests/golden/c2_shaped_steady_oracle.json: the FP64 oracle's steady state of a solve with the
velocity set and the physics of the single-instance FP64-vs-FP32 workload (HHLB(10;16) x HLB(7;8),
delta = 0.1, u_w = 0.2, omega = 0.66, A = 0.9) on 64 cells instead of 512, where the oracle reaches
the fixed point in minutes (the 512-cell solve takes it hours), and of the plain workload
(Nx = 32, HHLB(3;4) x HLB(3;4), delta = 1, u_w = 0.05, omega = 0.7).  Calls only oracle/; local
time steps (cap 64; the same fixed point as the global step) to a residual of 1e-12.  The fields
are stored for element-by-element comparison.

    python tests/golden/make_c2_shaped_steady.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.oracle import FIELD_NAMES, OracleProblem  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_shaped_steady_oracle.json")
TOL = 1e-12
CASES = {
    "c2_shaped_nx64_q16x8": dict(Qx=16, Qy=8, ncell=64, stretch_A=0.9, delta=0.1, uw=0.2, omega=0.66),
    "plain_nx32_q4x4": dict(Qx=4, Qy=4, ncell=32, stretch_A=0.0, delta=1.0, uw=0.05, omega=0.7),
}


def main():
    out = dict(source="FP64 oracle (oracle/), local time steps cap 64, residual < %g" % TOL, fields=list(FIELD_NAMES),
               cases={})
    for name, d in CASES.items():
        t0 = time.time()
        p = OracleProblem(d["Qx"], d["Qy"], d["ncell"], stretch_A=d["stretch_A"], delta=d["delta"], uw=d["uw"],
                          omega=d["omega"], local_dt_cap=64.0)
        phi, chi = p.init_state()
        steps, res = p.step(phi, chi, 20_000_000, 1000, TOL)
        assert res < TOL, res
        f = p.moments(phi, chi)
        out["cases"][name] = dict(params=d, steps=steps, residual=res, Pi=p.Pi(f), pxy_mean=p.mean_pxy(f),
                                  fields=f.tolist(), seconds=round(time.time() - t0, 1))
        print(name, steps, res, p.Pi(f), round(time.time() - t0, 1), flush=True)
    json.dump(out, open(OUT, "w"))


if __name__ == "__main__":
    main()

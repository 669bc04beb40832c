"""Writes tests/golden/pxy_steady_oracle.json: the FP64 oracle's steady states of the calibration
draws (hrlb_inputs.steady_calibration_draws), against which the P_xy error stop rule of the serving
loop is checked.  Calls only oracle/.  Each solve marches with local time steps (cap 64; the same
fixed point as the global step) to a residual of 1e-11.

    python tests/golden/make_pxy_steady.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from hrlb_inputs import steady_calibration_draws  # noqa: E402
from oracle.oracle import OracleProblem  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pxy_steady_oracle.json")
TOL = 1e-11


def main():
    rows = []
    for k, d in enumerate(steady_calibration_draws()):
        t0 = time.time()
        p = OracleProblem(d["Qx"], d["Qy"], d["ncell"], stretch_A=d["stretch_A"], delta=d["delta"], uw=d["uw"],
                          Tw=d["Tw"], Pr=d["Pr"], omega=d["omega"], local_dt_cap=64.0)
        phi, chi = p.init_state()
        steps, res = p.step(phi, chi, 5_000_000, 500, TOL)
        f = p.moments(phi, chi)
        rows.append(dict(draw=k, params=d, steps=steps, residual=res, pxy_mean=p.mean_pxy(f), Pi=p.Pi(f),
                         seconds=round(time.time() - t0, 1)))
        print(json.dumps(rows[-1]), flush=True)
        assert res < TOL, res
    json.dump(dict(source="FP64 oracle (oracle/), local time steps cap 64, residual < %g" % TOL, tol=TOL,
                   rows=rows), open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main()

"""Driving loop of the request server (hrlb_server_*) for a trace of timed arrivals.

Requests are handed to the server at their arrival times (seconds after the start of the trace); the
server is pumped whenever it holds work, and sleeps until the next arrival when it does not.  Every
scheduling decision and every step runs in libhrlb; this module only feeds arrivals and collects the
per-request records.
"""
from __future__ import annotations

import time

import numpy as np

from . import hrlb


def run_trace(server: "hrlb.Server", requests, arrivals, *, tol: float, max_steps: int,
              stop_rule: int = hrlb.HRLB_STOP_PXY, wall_limit_s: float = 600.0, local_dt_cap: float = 0.0,
              cfl: float = 0.5):
    """requests: dicts with Qx, Qy, ncell, stretch_A, delta, uw, Tw, Pr, omega, seed (hrlb_inputs
    draws); arrivals: seconds after the trace start.  Returns (records, totals): one record per
    request (arrival, admit and done times relative to the trace start, steps, status, Pi, the last
    estimate of the P_xy error rule) and the
    totals of the run (wall time, cell-velocity updates, rounds).  local_dt_cap > 1 runs every solve with
    local time steps (steady-state acceleration); cfl is the Courant number of the time step rule."""
    order = np.argsort(arrivals, kind="stable")
    t_start = server.clock()
    ids = {}
    nxt = 0
    units, rounds = 0.0, 0
    while True:
        now = server.clock() - t_start
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            k = int(order[nxt])
            d = requests[k]
            p = hrlb.make_params(delta=d["delta"], uw=d["uw"], ncell=d["ncell"], stretch_A=d["stretch_A"],
                                 Tw=d.get("Tw", 1.0), Pr=d.get("Pr", 2.0 / 3.0), omega=d["omega"],
                                 precision=server.precision, rounding=hrlb.HRLB_ROUND_STOCHASTIC,
                                 seed=d.get("seed", k), local_dt_cap=local_dt_cap, cfl=cfl)
            ids[k] = server.submit(d["Qx"], d["Qy"], p, tol=tol, max_steps=max_steps, stop_rule=stop_rule,
                                   arrival_s=t_start + float(arrivals[k]))
            nxt += 1
        st = server.pump()
        rounds += 1
        units += st.units
        if st.active == 0 and st.waiting == 0:
            if nxt >= len(order):
                break
            time.sleep(max(0.0, min(0.05, arrivals[order[nxt]] - (server.clock() - t_start))))
        if server.clock() - t_start > wall_limit_s:
            break
    wall = server.clock() - t_start
    records = []
    for k in range(len(requests)):
        if k not in ids:
            records.append(dict(index=k, state="not submitted"))
            continue
        info, _, _ = server.request(ids[k])
        state = {hrlb.HRLB_REQ_WAITING: "waiting", hrlb.HRLB_REQ_ACTIVE: "active", hrlb.HRLB_REQ_DONE: "done",
                 hrlb.HRLB_REQ_FAILED: "failed"}[info.state]
        rec = dict(index=k, state=state, status=info.status, steps=info.steps, Pi=info.Pi, pxy_err=info.pxy_err,
                   arrival=info.t_arrival - t_start, n_cells=info.n_cells, n_vel=info.n_vel, bytes=info.bytes)
        if info.t_admit >= 0:
            rec["admit"] = info.t_admit - t_start
        if info.t_done >= 0:
            rec["done"] = info.t_done - t_start
        records.append(rec)
    return records, dict(wall_s=wall, units=units, rounds=rounds)


def latency_summary(records):
    """Latencies of a trace.  time to steady = arrival -> result of a request that met its stop rule;
    a request that reached its step cap or failed never reached the target, so it counts as infinitely
    late in the percentiles over all requests (null when the percentile falls on one).  Also the same
    percentiles over the converged requests alone, arrival -> result and admission -> result over the
    finished ones, and the counts.  Percentiles are sample values (the smallest with at least q% of
    the samples at or below it), not interpolations."""
    done = [r for r in records if r.get("state") == "done"]
    conv = [r for r in done if r["status"] == hrlb.HRLB_OK]
    out = dict(requests=len(records), finished=len(done), converged=len(conv),
               capped=sum(1 for r in done if r["status"] == hrlb.HRLB_NOT_CONVERGED),
               failed=sum(1 for r in records if r.get("state") == "failed"),
               unfinished=len(records) - len(done) - sum(1 for r in records if r.get("state") == "failed"))
    def pct(x, q):
        # the smallest sample with at least q% of the samples at or below it (no interpolation)
        return float(np.percentile(x, q, method="inverted_cdf"))

    t_all = np.array([r["done"] - r["arrival"] if r in conv else np.inf for r in records])
    for q in (50, 99):
        v = pct(t_all, q) if len(t_all) else np.inf
        out[f"p{q}_time_to_steady_s"] = v if np.isfinite(v) else None
    if conv:
        t = np.array([r["done"] - r["arrival"] for r in conv])
        out.update(p50_time_to_steady_converged_s=pct(t, 50), p99_time_to_steady_converged_s=pct(t, 99))
    if done:
        a2r = np.array([r["done"] - r["arrival"] for r in done])
        d2r = np.array([r["done"] - r["admit"] for r in done])
        out.update(p50_arrival_to_result_s=pct(a2r, 50), p99_arrival_to_result_s=pct(a2r, 99),
                   p50_admit_to_result_s=pct(d2r, 50), p99_admit_to_result_s=pct(d2r, 99))
    return out

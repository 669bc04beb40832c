#!/usr/bin/env python3
"""Throughput of the half-range lattice Boltzmann Couette step on one MI355X.

A step is one full SSP-RK3 step (three stages: WENO-5 advection with diffuse walls, Shakhov
collision, stage update, FP64 moments) of every instance of the workload.  The default workload is
the ragged batch of 512 Couette instances drawn with seed 0 (delta = 10^U(-2,2), u_w ~ U(0.01,0.5),
omega ~ U(0.5,1), Nx in {64..1024}, Qx in {4,8,16,32}, Qy in {4,8,12}, tanh stretching A = 0.9),
with FP32 populations (stochastic rounding) and FP64 moments, advanced by shared launches.

Prints one JSON line.  --gpus above 1 is refused: this solver runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Batch workloads run the batch plan: each instance asks for rows of tile_vpt = the largest divisor
# of Q_y up to 16 that still fills a group's 16 rows (the library's default rows hold at most 8
# velocities), and for one lane per cell in the per-cell kernel (the default is two).  With
# thousands of tiles and hundreds of thousands of cells per launch, longer rows spread the per-tile
# work over more velocities and single lanes halve the per-cell blocks; the serving loop's smaller
# batches keep the defaults, which fill the GPU with more tiles and blocks.
WORKLOADS = {
    "couette_batch512_ragged_fp32": dict(kind="batch", precision=1, rounding=1, rows="long", lanes=1),
    "couette_batch512_ragged_fp64": dict(kind="batch", precision=0, rounding=0, rows="long", lanes=1),
    "couette_nx512_q16x8_fp64": dict(kind="single", name="couette_nx512_q16x8", precision=0, rounding=0),
    # the plain method in FP64, one instance, run to a residual below 1e-10: time to steady
    "couette_nx32_q4x4_fp64_steady": dict(kind="steady", name="couette_nx32_q4x4_fp64", precision=0, rounding=0,
                                          tol=1e-10, check_every=100, max_steps=1000000),
    "couette_nx512_q16x8_fp32": dict(kind="single", name="couette_nx512_q16x8", precision=1, rounding=1),
    "couette_nx2048_q80x20_fp32": dict(kind="single", name="couette_nx2048_q80x20", precision=1, rounding=1),
    "couette_nx2048_q80x20_fp64": dict(kind="single", name="couette_nx2048_q80x20", precision=0, rounding=0),
    # the same flows as their right halves (point symmetry of Sec. II): n_cells/2 cells per instance,
    # one diffuse wall, half the updates per step
    "couette_batch512_ragged_half_fp32": dict(kind="batch", precision=1, rounding=1, half=True, rows="long",
                                              lanes=1),
    "couette_nx512_q16x8_half_fp32": dict(kind="single", name="couette_nx512_q16x8", precision=1, rounding=1,
                                          half=True),
    # serving: 64 solves drawn like the ragged batch with Nx up to 2048 (seed 1), Poisson arrivals at
    # 200 requests/s (seed 2), FP32 storage; each stops when its P_xy drift rate falls below 2e-6 per
    # unit time or after 100k steps
    "couette_serve_poisson200": dict(kind="serve", precision=1, rounding=1, requests=64, rate=200.0,
                                     tol=2e-6, max_steps=100000, check_every=1000),
    # the same trace with local time steps (steady-state acceleration, cap 64)
    "couette_serve_poisson200_lts": dict(kind="serve", precision=1, rounding=1, requests=64, rate=200.0,
                                         tol=2e-6, max_steps=100000, check_every=1000, local_dt_cap=64.0),
    # the serving metric: each solve stops once the estimated remaining error of its mean P_xy is below
    # 3e-6 on two checks (the rule that keeps every oracle-checked calibration draw within 1e-5 of the
    # oracle's steady state), local time steps, Courant number 1 (the steady state does not depend on
    # the time step; the oracle reaches the same one at CFL 1), at most 1M steps; the default run serves
    # the first 32 requests of this trace next to the batch
    "couette_serve_poisson200_pxyerr": dict(kind="serve", precision=1, rounding=1, requests=64, rate=200.0,
                                            tol=3e-6, stop_rule=2, max_steps=1000000, check_every=250,
                                            local_dt_cap=64.0, cfl=1.0),
    # the quadrature-convergence claim of Sec. IV in its own setting: half channel, A = 0.98,
    # u_w = sqrt(2 K_B T_w/m), delta in {10, 1, 0.1}; the production models HHLB(6;7) x HLB(6;7)
    # (delta = 10, 1) and HHLB(10;16) x HLB(6;7) (delta = 0.1) on S = 16 cells against the reference
    # HHLB(10;50) x HLB(6;7) on S = 48 cells, every solve in FP64 to a P_xy drift rate of tol per unit
    # time, served together; mu ~ T^0.66 stands in for the helium tables
    "couette_paper_convergence": dict(kind="study", tol=1e-7, max_steps=4000000, check_every=2000),
    # the same six solves with local time steps (steady-state acceleration, cap 64)
    "couette_paper_convergence_lts": dict(kind="study", tol=1e-7, max_steps=4000000, check_every=2000,
                                          local_dt_cap=64.0),
    # and with each solve's plan from the autotuner
    "couette_paper_convergence_lts_tuned": dict(kind="study", tol=1e-7, max_steps=4000000, check_every=2000,
                                                local_dt_cap=64.0, tune=True),
}


def _instances(spec):
    from hrlb_inputs import batch_draws, case

    if spec["kind"] == "batch":
        return batch_draws(512, seed=0)
    d = case(spec["name"])
    d["seed"] = 12345
    return [d]


def long_row_vpt(Qx: int, Qy: int) -> int:
    """Velocities per stage-kernel row of the long-row plan: the largest divisor of Qy up to 16 that
    leaves at least 16 rows (2 Qx Qy / vpt >= 16)."""
    return max(d for d in range(1, min(Qy, 16) + 1) if Qy % d == 0 and 2 * Qx * Qy // d >= 16)


def _build(spec, insts, tune: bool, tile_vpt: int = 0, cell_lanes: int = 0, rows: str = "default"):
    """Cases of the workload; a single instance gets its stage-kernel tiling from the autotuner.
    tile_vpt / cell_lanes > 0 impose a plan on every instance (where admissible); rows="long" asks
    every instance for the long-row plan."""
    from paper_1810_07803_amd import hrlb

    quads, cases, tuned = {}, [], None
    for d in insts:
        key = (d["Qx"], d["Qy"])
        if key not in quads:
            quads[key] = hrlb.Quadrature(d["Qx"], d["Qy"])
        half = bool(spec.get("half"))
        kw = dict(delta=d["delta"], uw=d["uw"], ncell=d["ncell"] // 2 if half else d["ncell"],
                  stretch_A=d["stretch_A"], Tw=d.get("Tw", 1.0), Pr=d.get("Pr", 2.0 / 3.0), omega=d["omega"],
                  precision=spec["precision"], rounding=spec["rounding"], seed=d.get("seed", 0),
                  half_channel=int(half))
        if cell_lanes > 0:
            kw["cell_lanes"] = cell_lanes
        if tile_vpt > 0 and d["Qy"] % tile_vpt == 0:
            kw["tile_vpt"] = tile_vpt
        elif rows == "long":
            kw["tile_vpt"] = long_row_vpt(d["Qx"], d["Qy"])
        if tune and len(insts) == 1:
            tuned = hrlb.tune_plan(quads[key], hrlb.make_params(**kw), n_steps=10)
            kw["tile_vpt"], kw["cell_lanes"] = tuned[0], tuned[1]
        cases.append(hrlb.Case(quads[key], hrlb.make_params(**kw)))
    return quads, cases, hrlb.Batch(cases), tuned


def _cpu_baseline(insts, budget_s: float, half: bool = False):
    """The oracle as it stands, on a bounded sample of the same workload (host cores, OpenMP).  The
    sample is the instances at the work-weighted sixths of the workload (instances ordered by cell x
    velocity count, the one holding the midpoint of each sixth of the total), so that its mix of sizes
    is the mix the batch's updates come from; every sampled instance runs the same number of steps."""
    from oracle.oracle import OracleProblem, num_threads

    if len(insts) <= 6:
        sample = list(insts)
    else:
        size = [d["ncell"] * 2 * d["Qx"] * d["Qy"] for d in insts]
        order = sorted(range(len(insts)), key=lambda k: size[k])
        total = float(sum(size))
        sample, acc, want = [], 0.0, [(2 * i + 1) / 12.0 * total for i in range(6)]
        for k in order:
            acc += size[k]
            while want and acc >= want[0]:
                sample.append(insts[k])
                want.pop(0)
    probs = []
    for d in sample:
        probs.append(OracleProblem(d["Qx"], d["Qy"], d["ncell"] // 2 if half else d["ncell"],
                                   stretch_A=d["stretch_A"], delta=d["delta"], uw=d["uw"], omega=d["omega"],
                                   half_channel=half))
    # one calibration step each, then as many steps as fit in the budget
    t0 = time.perf_counter()
    states = []
    for p in probs:
        phi, chi = p.init_state()
        p.step(phi, chi, 1)
        states.append((phi, chi))
    t_cal = time.perf_counter() - t0
    steps = max(1, int(budget_s / max(t_cal, 1e-3)))
    t0 = time.perf_counter()
    units = 0
    for p, (phi, chi) in zip(probs, states):
        p.step(phi, chi, steps)
        units += p.nv * p.ncell * steps
    dt = time.perf_counter() - t0
    return {"value": units / dt, "unit": "cell·velocity updates/s", "cores": num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle, {len(sample)} instances at the work-weighted sixths of the workload "
                      f"(cells x velocities {sorted(p.nv * p.ncell for p in probs)}), {steps} steps each "
                      f"({units} cell·velocity updates in {dt:.1f} s)"}


def _serve_trace(args, spec, n_requests, wall_limit_s):
    """Serves a Poisson trace of n_requests solves drawn like the ragged batch with Nx up to 2048 (seed 1,
    arrivals seed 2) with continuous batching; returns (summary, totals)."""
    from hrlb_inputs import batch_draws, poisson_arrivals
    from paper_1810_07803_amd import hrlb, serve

    reqs = batch_draws(n_requests, seed=1, nx_choices=(64, 128, 256, 512, 1024, 2048))
    arrivals = poisson_arrivals(n_requests, spec["rate"], seed=2)
    arrivals = arrivals - arrivals[0]
    srv = hrlb.Server(args.arena_mib << 20, max_active=256, check_every=spec["check_every"], max_bypass=4,
                      precision=spec["precision"])
    # warm-up (kernel loading, velocity-set construction) on one small solve, untimed
    srv.submit(4, 4, hrlb.make_params(delta=1.0, uw=0.1, ncell=64, precision=spec["precision"], rounding=1),
               tol=1.0, max_steps=spec["check_every"])
    while srv.pump().active:
        pass
    print(f"# serving {len(reqs)} requests", file=sys.stderr, flush=True)
    records, tot = serve.run_trace(srv, reqs, arrivals, tol=spec["tol"], max_steps=spec["max_steps"],
                                   stop_rule=spec.get("stop_rule", hrlb.HRLB_STOP_PXY), wall_limit_s=wall_limit_s,
                                   local_dt_cap=spec.get("local_dt_cap", 0.0), cfl=spec.get("cfl", 0.5))
    summ = serve.latency_summary(records)
    summ["solves_per_s"] = summ["finished"] / tot["wall_s"]
    summ["updates_per_s"] = tot["units"] / tot["wall_s"]
    summ["rounds"] = tot["rounds"]
    summ["wall_s"] = tot["wall_s"]
    srv.free()
    return summ, tot, reqs


def _stop_desc(spec):
    from paper_1810_07803_amd import hrlb

    rule = {hrlb.HRLB_STOP_PXY: "pxy_drift", hrlb.HRLB_STOP_PXY_ERR: "pxy_error_estimate",
            hrlb.HRLB_STOP_RESIDUAL: "residual"}[spec.get("stop_rule", hrlb.HRLB_STOP_PXY)]
    return {"rule": rule, "tol": spec["tol"], "max_steps": spec["max_steps"], "check_every": spec["check_every"]}


def _serve_main(args, spec):
    """Serving workload: requests arrive on a Poisson trace and are served with continuous batching."""
    summ, tot, reqs = _serve_trace(args, spec, spec["requests"], args.serve_wall_s)
    out = {
        "metric": "cell·velocity updates/s",
        "value": tot["units"] / tot["wall_s"],
        "unit": "cell·velocity updates/s",
        "n_gpus": 1, "steps": tot["rounds"], "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "moments_dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "requests": len(reqs), "arrival_rate_per_s": spec["rate"],
                   "stop": _stop_desc(spec),
                   "arena_mib": args.arena_mib, "local_dt_cap": spec.get("local_dt_cap", 0.0),
                   "cfl": spec.get("cfl", 0.5), "parallelism": "single GPU, continuous batching"},
        "serving": summ,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def _study_main(args, spec):
    """Sec. IV convergence study: every solve through the request server, Pi of each production model
    against the reference model at the same delta."""
    from paper_1810_07803_amd import hrlb

    uw = math.sqrt(2.0)
    runs = []
    for delta in (10.0, 1.0, 0.1):
        Qx, Nx = (7, 6) if delta >= 1.0 else (16, 10)
        runs.append(dict(delta=delta, role="production", model=f"HHLB({Nx};{Qx})xHLB(6;7)", Qx=Qx, Nx=Nx, S=16))
        runs.append(dict(delta=delta, role="reference", model="HHLB(10;50)xHLB(6;7)", Qx=50, Nx=10, S=48))
    srv = hrlb.Server(args.arena_mib << 20, max_active=16, check_every=spec["check_every"], max_bypass=4,
                      precision=hrlb.HRLB_FP64)
    t0 = time.perf_counter()
    ids = []
    for r in runs:
        kw = dict(delta=r["delta"], uw=uw, ncell=r["S"], stretch_A=0.98, omega=0.66, precision=hrlb.HRLB_FP64,
                  half_channel=1, local_dt_cap=spec.get("local_dt_cap", 0.0))
        if spec.get("tune"):
            # these solves are small enough to be latency bound: the autotuner's plan per solve
            q = hrlb.Quadrature(r["Qx"], 7, r["Nx"], 6)
            kw["tile_vpt"], kw["cell_lanes"], _ = hrlb.tune_plan(q, hrlb.make_params(**kw), n_steps=20)
            r["plan"] = [kw["tile_vpt"], kw["cell_lanes"]]
        ids.append(srv.submit(r["Qx"], 7, hrlb.make_params(**kw), tol=spec["tol"], max_steps=spec["max_steps"],
                              Nx=r["Nx"], Ny=6))
    units, last = 0.0, t0
    while True:
        st = srv.pump()
        units += st.units
        now = time.perf_counter()
        if now - last > 10.0:
            print(f"# {now - t0:.0f} s: {st.active} active, {st.done} done, {st.steps} steps in the last round",
                  file=sys.stderr, flush=True)
            last = now
        if st.active == 0 and st.waiting == 0:
            break
        if now - t0 > args.serve_wall_s:
            print("# wall-clock limit reached", file=sys.stderr, flush=True)
            break
    wall = time.perf_counter() - t0
    results = []
    for r, rid in zip(runs, ids):
        info, _, _ = srv.request(rid)
        results.append(dict(r, state=int(info.state), status=int(info.status), steps=int(info.steps),
                            Pi=info.Pi, pxy_drift=info.pxy_drift, sim_time=info.sim_time,
                            time_to_steady_s=(info.t_done - info.t_admit) if info.t_done >= 0 else None))
    errs = {}
    for k in range(0, len(results), 2):
        prod, ref = results[k], results[k + 1]
        errs[f"delta={prod['delta']:g}"] = prod["Pi"] / ref["Pi"] - 1.0
    out = {
        "metric": "cell·velocity updates/s",
        "value": units / wall,
        "unit": "cell·velocity updates/s",
        "n_gpus": 1, "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "moments_dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "solves": len(runs), "half_channel": True, "stretch_A": 0.98,
                   "local_dt_cap": spec.get("local_dt_cap", 0.0), "tuned_plans": bool(spec.get("tune")),
                   "u_w": uw, "omega": 0.66, "stop": {"rule": "pxy_drift", "tol": spec["tol"],
                                                      "check_every": spec["check_every"]},
                   "parallelism": "single GPU, continuous batching"},
        "study": {"runs": results, "Pi_rel_err_production_vs_reference": errs,
                  "claim": "production models within 0.1% of the reference (Sec. IV)", "wall_s": wall,
                  "solves_per_s": len(runs) / wall},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def _steady_main(args, spec):
    """One instance run to steady state with hrlb_run_to_steady (residual rule), timed end to end."""
    from hrlb_inputs import case
    from paper_1810_07803_amd import hrlb

    d = case(spec["name"])
    q = hrlb.Quadrature(d["Qx"], d["Qy"])
    params = hrlb.make_params(delta=d["delta"], uw=d["uw"], ncell=d["ncell"], stretch_A=d["stretch_A"],
                              omega=d["omega"], precision=spec["precision"], rounding=spec["rounding"])
    # warm-up: kernel loading and one short run on a separate case
    hrlb.Case(q, params).step(10)
    c = hrlb.Case(q, params)
    t0 = time.perf_counter()
    st, info = c.run_to_steady(spec["tol"], spec["max_steps"], spec["check_every"])
    wall = time.perf_counter() - t0
    f, x, pi, shear = c.moments()
    units = c.nv * c.ncell * info.steps
    out = {
        "metric": "cell·velocity updates/s",
        "value": units / wall,
        "unit": "cell·velocity updates/s",
        "n_gpus": 1, "steps": int(info.steps), "warmup": 10, "ms_per_step": wall / max(1, info.steps) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if spec["precision"] == 0 else "f32", "moments_dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "case": d, "stop": {"rule": "residual", "tol": spec["tol"],
                                                                  "check_every": spec["check_every"]},
                   "parallelism": "single GPU, one instance"},
        "steady": {"status": int(st), "steps": int(info.steps), "residual": info.residual,
                   "time_to_steady_s": wall, "solves_per_s": 1.0 / wall, "Pi": pi, "mass_drift": info.mass_drift,
                   "wall_shear": [float(shear[0]), float(shear[1])]},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="couette_batch512_ragged_fp32", choices=sorted(WORKLOADS))
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the tiling autotuner for single instances")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="steps per captured HIP graph (0 launches every kernel directly)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (calibrates HBM byte counters)")
    ap.add_argument("--streams", type=int, default=3,
                    help="parts of the batch advanced on separate streams (1-4; 3 is the library's default for "
                    "batches of at least 2e7 units)")
    ap.add_argument("--cell-lanes", type=int, default=0, help="lanes per cell of the per-cell kernel for every "
                    "instance (0 = the workload's plan: 1 for the batches, else each instance's automatic choice)")
    ap.add_argument("--tile-vpt", type=int, default=0, help="velocities per stage-kernel row for every instance "
                    "whose Qy it divides (0 = automatic)")
    ap.add_argument("--rows", choices=("default", "long"), default=None,
                    help="stage-kernel rows of every instance: the library default (at most 8 velocities) or the "
                    "long-row plan (up to 16); default: the workload's own choice")
    ap.add_argument("--arena-mib", type=int, default=4096, help="serving: device arena for resident solves")
    ap.add_argument("--serve-wall-s", type=float, default=240.0, help="serving: wall-clock limit of the trace")
    ap.add_argument("--serve-requests", type=int, default=32,
                    help="default workload: requests of the serving trace run after the batch (0 skips it)")
    ap.add_argument("--serve-leg-wall-s", type=float, default=180.0,
                    help="default workload: wall-clock limit of that serving trace")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not supported "
              "(independent instances would shard by instance, see the design notes)", file=sys.stderr)
        return 2

    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    spec = WORKLOADS[args.workload]
    if spec["kind"] == "serve":
        return _serve_main(args, spec)
    if spec["kind"] == "study":
        return _study_main(args, spec)
    if spec["kind"] == "steady":
        return _steady_main(args, spec)
    insts = _instances(spec)
    print(f"# building {len(insts)} instance(s) of {args.workload}", file=sys.stderr, flush=True)
    rows = args.rows or spec.get("rows", "default")
    lanes = args.cell_lanes if args.cell_lanes > 0 else spec.get("lanes", 0)
    quads, cases, batch, tuned = _build(spec, insts, tune=not args.no_tune, tile_vpt=args.tile_vpt,
                                        cell_lanes=lanes, rows=rows)
    units = sum(c.nv * c.ncell for c in cases)
    from paper_1810_07803_amd import hrlb as _h

    # the stage kernel advances the cases of the tiled path; the small path's cases run one launch of
    # their own per block of steps
    tiled_units = sum(c.nv * c.ncell for c in cases if c.kernel_path() == _h.HRLB_PATH_TILED)
    n_small = sum(1 for c in cases if c.kernel_path() == _h.HRLB_PATH_SMALL)
    batch.set_graph_steps(args.graph_steps)
    batch.set_streams(args.streams)
    stream = torch.cuda.current_stream()

    batch.step(args.warmup)
    torch.cuda.synchronize()
    print(f"# warmup done, timing {args.steps} steps", file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    batch.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    value = units / (ms_per_step * 1e-3)

    # kernel roofline on whole-batch launches that have the GPU to themselves (one stream), so that a
    # launch's bytes and duration belong to the same work; the timed steps above use args.streams
    batch.set_streams(1)
    stage_ms, cell_ms = batch.profile(args.profile_steps)
    batch.set_streams(args.streams)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    es = 4 if spec["precision"] == 1 else 8
    # algorithmic bytes per stage launch: read f_in and write f_out (both dists) in every stage,
    # plus f^n in stages 2 and 3: (2 + 3 + 3)/3 passes of 2 dists per unit on average
    bytes_per_unit = es * 2 * (2 + 3 + 3) / 3.0
    achieved = tiled_units * bytes_per_unit / (stage_ms * 1e-3) / 1e9
    from paper_1810_07803_amd import profiling

    traffic = profiling.load_traffic(os.path.join(ROOT, "profiles", f"{args.workload}_stage_kernel_traffic.txt"))
    tname = "float" if es == 4 else "double"
    valu = profiling.load_sq(os.path.join(ROOT, "profiles", f"{args.workload}_sq_counters.md"),
                             [f"stage_kernel<{tname}, {m}>" for m in (1, 2, 3)])
    # the method floor: a whole step reads and writes phi and chi once in the storage precision
    # (2 x 2 x es bytes per unit) at the HBM peak
    floor_frac = value * 4 * es / (HBM_PEAK_GBS * 1e9)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "stage_kernel<%s, 1..3> (the three stages of a step)" % ("float" if es == 4 else "double"),
                "kernel_ms": round(stage_ms, 4), "cell_kernel_ms": round(cell_ms, 4),
                "bytes_per_unit_per_launch": bytes_per_unit, "units_per_launch": tiled_units,
                "small_path_instances": n_small,
                "launches": "whole batch on one stream",
                "method_floor_frac": round(floor_frac, 4),
                "method_floor_bytes_per_unit_per_step": 4 * es,
                # VALU instructions per unit and issue share of the step kernels from the SQ-counter
                # profile of the same kernels (null once the kernels have changed): the kernel is bound
                # by VALU issue, not by HBM
                "valu": valu}

    cpu = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = _cpu_baseline(insts, args.cpu_seconds, half=bool(spec.get("half")))

    # the serving half of the metric: solves/s and time to steady at a fixed P_xy error, on a bounded trace
    serving = None
    n_inst = len(cases)
    if args.serve_requests > 0 and args.workload == "couette_batch512_ragged_fp32":
        batch.free()
        for c in cases:
            c.free()
        del cases, batch
        sspec = WORKLOADS["couette_serve_poisson200_pxyerr"]
        summ, _, reqs = _serve_trace(args, sspec, args.serve_requests, args.serve_leg_wall_s)
        serving = dict(summ, workload="couette_serve_poisson200_pxyerr", requests=len(reqs),
                       arrival_rate_per_s=sspec["rate"], stop=_stop_desc(sspec),
                       local_dt_cap=sspec["local_dt_cap"], cfl=sspec["cfl"], dtype="f32", moments_dtype="f64",
                       target="mean P_xy within 1e-5 of the steady state")

    out = {
        "metric": "cell·velocity updates/s",
        "value": value,
        "unit": "cell·velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if es == 4 else "f64",
        "moments_dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "instances": n_inst, "units_per_step": units,
                   "half_channel": bool(spec.get("half")),
                   "graph_steps": args.graph_steps, "streams": args.streams, "rows": rows, "cell_lanes": lanes,
                   "tuned_plan": {"tile_vpt": tuned[0], "cell_lanes": tuned[1]} if tuned else None,
                   "parallelism": "single GPU, instances batched per launch"},
        "wall_s_timed": wall,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

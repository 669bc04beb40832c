"""Summaries of rocprofv3 output for the solver's kernels (tracing/profiling support).

* ``stats``: the kernel table of a ``rocprofv3 --kernel-trace --stats --output-format csv`` run.
* ``sq``: instructions per cell-velocity unit and the VALU issue share per kernel (SQ counters).
* ``traffic``: HBM bytes per dispatch of one kernel from two counter runs (``--pmc FETCH_SIZE`` and
  ``--pmc WRITE_SIZE``, values in KiB per dispatch), each scaled by what the same counter reads for
  the largest plain device copy in the same run (``bench.py --copy-probe-mib N`` issues one of a
  known size).  The summary records a digest of the kernel sources (their code with comments
  removed and white space collapsed, so that an edit of a comment keeps it); ``load_traffic``
  returns the figures only while the sources still have that digest.

Command line:
    python -m paper_1810_07803_amd.profiling stats <kernel_stats.csv> [command...]
    python -m paper_1810_07803_amd.profiling traffic <fetch.csv> <write.csv> <kernel-substring> <probe-MiB> [command...]
    python -m paper_1810_07803_amd.profiling sq <counter_collection.csv> <units-per-launch> [command...]
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/hrlb_kernels.hip", "csrc/hrlb_internal.h", "csrc/hrlb_math.h", "csrc/hrlb_plan.h", "csrc/hrlb_host.cpp")


_TOKENS = re.compile(r'"(?:\\.|[^"\\])*"|(?:\s|//[^\n]*|/\*.*?\*/)+', re.S)


def code_only(text: str) -> str:
    """C/C++ source with every run of white space and comments made one space (string literals
    kept as written)."""
    return _TOKENS.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", text).strip()


def source_digest(root: str = HERE) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(root, rel), encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def stats(path: str, command: str = "") -> str:
    rows = list(csv.DictReader(open(path)))
    out = []
    if command:
        out.append(f"command: {command}")
    out.append(f"kernel source digest: {source_digest()}")
    out.append("")
    out.append("| kernel | calls | total ms | average us | min us | max us | % |")
    out.append("|---|---:|---:|---:|---:|---:|---:|")
    for r in rows:
        name = r["Name"].replace("|", "/")
        out.append("| %s | %s | %.3f | %.2f | %.2f | %.2f | %.1f |" % (
            name[:90], r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(out) + "\n"


def _per_dispatch(path: str, counter: str):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]


def traffic(fetch_csv: str, write_csv: str, kernel: str, probe_mib: float, command: str = "") -> str:
    """kernel: a substring of the kernel names, or several separated by ';' (the dispatches of all of
    them are averaged: the three stage variants of a step give the mean per stage launch)."""
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    known_kib = probe_mib * 1024.0
    # calibration: the copy dispatch that wrote the most bytes is the probe copy
    cal_w = max(v for n, v in write if "copy" in n.lower() or "elementwise" in n.lower())
    cal_f = max(v for n, v in fetch if "copy" in n.lower() or "elementwise" in n.lower())
    f_scale, w_scale = known_kib / cal_f, known_kib / cal_w
    names = [k for k in kernel.split(";") if k]
    kf = [v for n, v in fetch if any(k in n for k in names)]
    kw = [v for n, v in write if any(k in n for k in names)]
    f_kib = sum(kf) / len(kf)
    w_kib = sum(kw) / len(kw)
    tb = (f_kib * f_scale + w_kib * w_scale) * 1024.0
    lines = []
    if command:
        lines.append(f"command: {command}")
    lines += [
        f"kernel: {kernel}",
        f"kernel_source_digest: {source_digest()}",
        f"dispatches_fetch: {len(kf)}",
        f"dispatches_write: {len(kw)}",
        f"fetch_kib_per_dispatch: {f_kib:.1f}",
        f"write_kib_per_dispatch: {w_kib:.1f}",
        f"probe_copy_mib: {probe_mib}",
        f"probe_fetch_kib: {cal_f:.1f}",
        f"probe_write_kib: {cal_w:.1f}",
        f"fetch_scale: {f_scale:.4f}",
        f"write_scale: {w_scale:.4f}",
        f"traffic_bytes_per_dispatch: {tb:.0f}",
    ]
    return "\n".join(lines) + "\n"


def sq(path: str, units_per_launch: float, command: str = "") -> str:
    """Per-kernel table of a ``--pmc SQ_WAVES SQ_INSTS_VALU ...`` run: dispatches, mean duration, VALU,
    LDS and SALU instructions per cell-velocity unit of the launch (wave instructions x 64 lanes /
    units), and the VALU issue share: SQ_INSTS_VALU x 4 cycles (a wave64 VALU instruction on a 16-lane
    SIMD) over the 1024 SIMDs x the duration x 2.4 GHz."""
    rows = list(csv.DictReader(open(path)))
    agg, disp, dur = {}, {}, {}
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        if "hrlb::" not in name:
            continue
        a = agg.setdefault(name, {})
        a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        disp.setdefault(name, set()).add(r["Dispatch_Id"])
        dur.setdefault(name, {})[r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = []
    if command:
        out.append(f"command: {command}")
    out.append(f"kernel source digest: {source_digest()}")
    out.append(f"units per launch: {units_per_launch:.0f}")
    out.append("")
    out.append("| kernel | dispatches | mean us | VALU/unit | LDS/unit | SALU/unit | VALU issue share |")
    out.append("|---|---:|---:|---:|---:|---:|---:|")
    for name in sorted(agg):
        n = len(disp[name])
        a = agg[name]
        d_ns = sum(dur[name].values()) / n
        per = lambda c: a.get(c, 0.0) / n * 64.0 / units_per_launch
        share = a.get("SQ_INSTS_VALU", 0.0) / n * 4.0 / (1024.0 * d_ns * 2.4)
        out.append("| %s | %d | %.1f | %.1f | %.1f | %.1f | %.3f |" % (
            name.replace("hrlb::", ""), n, d_ns / 1e3, per("SQ_INSTS_VALU"), per("SQ_INSTS_LDS"),
            per("SQ_INSTS_SALU"), share))
    return "\n".join(out) + "\n"


def load_traffic(path: str):
    """Traffic bytes per dispatch from a summary, or None if absent or the kernels have changed."""
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_digest") != source_digest():
        return None
    try:
        return float(kv["traffic_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def load_sq(path: str, kernels):
    """From an SQ-counter summary: the VALU instructions per unit and the VALU issue share averaged over
    the given kernels weighted by their dispatch counts, or None if absent or the kernels have changed."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel source digest: (\w+)", text)
    if not m or m.group(1) != source_digest():
        return None
    rows = {}
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] in kernels:
            rows[cells[0]] = (int(cells[1]), float(cells[3]), float(cells[6]))
    if not rows:
        return None
    n = sum(r[0] for r in rows.values())
    return {"valu_per_unit": round(sum(r[0] * r[1] for r in rows.values()) / n, 1),
            "valu_issue_share": round(sum(r[0] * r[2] for r in rows.values()) / n, 3)}


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        sys.stdout.write(stats(sys.argv[2], " ".join(sys.argv[3:])))
    elif mode == "traffic":
        sys.stdout.write(traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), " ".join(sys.argv[6:])))
    elif mode == "sq":
        sys.stdout.write(sq(sys.argv[2], float(sys.argv[3]), " ".join(sys.argv[4:])))
    else:
        raise SystemExit(__doc__)

"""Kernel statistics of rocprofv3 output: a kernel trace cut to a timed
window, and HBM bytes per launch from counter runs.

window: rocprofv3 --kernel-trace --output-format csv writes one row per
dispatch with start and end timestamps.  bench.py --trace-window FILE records,
for each timed run, the host clocks (CLOCK_MONOTONIC and CLOCK_BOOTTIME, ns) at
the synchronised start and end of its timed steps.  The dispatches that start
inside one such window are grouped by kernel name and launch grid (the levels
of a hierarchy may share both).  Within a group, launches that take less than
a fifth of the group's 90th-percentile duration are counted apart as short
launches: coarser levels launched with the same grid, and the iterations of a
captured Krylov chunk that begin after convergence and return at once.  The
averages over the remaining launches are the per-launch figures a roofline
may use.

traffic: two rocprofv3 --pmc runs of one command (FETCH_SIZE, then
WRITE_SIZE; KiB per dispatch) give the HBM bytes of the last N dispatches of a
kernel (bench.py's back-to-back roofline launches come last).  Each counter is
scaled by what it reads for a plain device copy of known size (bench.py
--calibrate-copy, profiled the same two ways), and the result is written as
JSON keyed by the sources' hash, so that bench.py uses it only while the
kernels are unchanged.

    python -m paper_2204_07019_amd.trace_window window TRACE.csv WINDOW.json [--leg NAME] [--top N]
    python -m paper_2204_07019_amd.trace_window traffic --fetch F.csv --write W.csv --calib-fetch CF.csv \\
        --calib-write CW.csv --family NAME --kernel-regex RE --last N --algorithmic BYTES --out JSON [--command CMD]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys
from collections import defaultdict

SHORT_FRAC = 0.2
COPY_BYTES = 1 << 30   # bench.py --calibrate-copy: 2^27 FP64 values per copy
HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_sources_sha() -> str:
    """Hash of the HIP sources (csrc/*): counter figures hold for these only."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------- window

def load_trace(path):
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            grid = (int(r["Grid_Size_X"]), int(r["Grid_Size_Y"]), int(r["Grid_Size_Z"]))
            wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"], grid, wg))
    rows.sort()
    return rows


def pick_clock(rows, win):
    """The host clock whose window holds the most dispatch starts (the one the
    trace's timestamps follow)."""
    best, best_n = None, -1
    for clock, (a, b) in win.items():
        n = sum(1 for r in rows if a <= r[0] <= b)
        if n > best_n:
            best, best_n = clock, n
    return best, best_n


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return 0.0
    k = min(len(xs) - 1, max(0, int(round(q * (len(xs) - 1)))))
    return xs[k]


def window_stats(rows, a, b):
    groups = defaultdict(list)
    for s, e, name, grid, wg in rows:
        if a <= s <= b:
            groups[(name, grid, wg)].append(e - s)
    total = sum(sum(v) for v in groups.values())
    out = []
    for (name, grid, wg), durs in groups.items():
        p90 = percentile(durs, 0.9)
        full = [d for d in durs if d >= SHORT_FRAC * p90]
        short = [d for d in durs if d < SHORT_FRAC * p90]
        out.append(dict(name=name, grid=grid, workgroup=wg, calls=len(durs), short_calls=len(short),
                        total_ns=sum(durs), full_avg_ns=(sum(full) / len(full)) if full else 0.0,
                        short_avg_ns=(sum(short) / len(short)) if short else 0.0,
                        frac=sum(durs) / total if total else 0.0))
    out.sort(key=lambda d: -d["total_ns"])
    return out, total


def by_name(stats):
    agg = defaultdict(lambda: [0, 0])
    for d in stats:
        agg[d["name"]][0] += d["total_ns"]
        agg[d["name"]][1] += d["calls"]
    return sorted(((k, v[0], v[1]) for k, v in agg.items()), key=lambda t: -t[1])


def short_name(name, width=90):
    return name if len(name) <= width else name[:width - 3] + "..."


def cmd_window(args):
    rows = load_trace(args.trace)
    wins = json.load(open(args.window))
    if args.leg not in wins:
        sys.exit(f"no window named {args.leg!r} in {args.window} (have {sorted(wins)})")
    w = wins[args.leg]
    clock, n = pick_clock(rows, {k: w[k] for k in ("monotonic", "boottime")})
    a, b = w[clock]
    stats, total = window_stats(rows, a, b)
    steps = w.get("steps", 1)
    wall = (b - a) * 1e-9
    print(f"window {args.leg!r}: {steps} timed steps, {wall * 1e3:.1f} ms wall on {clock}, {n} dispatches, "
          f"kernel busy {total * 1e-6:.1f} ms ({total * 1e-9 / wall * 100:.1f} % of the window; "
          f"above 100 % where streams overlap)\n")
    print("By kernel and launch grid (short = launches under a fifth of the group's 90th-percentile duration):\n")
    print("| kernel | grid | calls | short | total ms | % | avg us (full) | avg us (short) |")
    print("|---|---|---:|---:|---:|---:|---:|---:|")
    for d in stats[:args.top]:
        print(f"| `{short_name(d['name'])}` | {d['grid'][0]}x{d['grid'][1]}x{d['grid'][2]} | {d['calls']} | "
              f"{d['short_calls']} | {d['total_ns'] * 1e-6:.2f} | {d['frac'] * 100:.1f} | "
              f"{d['full_avg_ns'] * 1e-3:.1f} | {d['short_avg_ns'] * 1e-3:.1f} |")
    print("\nBy kernel name (all grids):\n")
    print("| kernel | calls | total ms | % |")
    print("|---|---:|---:|---:|")
    for name, t, c in by_name(stats)[:args.top]:
        print(f"| `{short_name(name)}` | {c} | {t * 1e-6:.2f} | {t / total * 100:.1f} |")
    return 0


# ---------------------------------------------------------------- traffic

def counter_values(path, counter, kernel_re=None):
    """Per-dispatch values of one counter (summed over the CSV's rows of a
    dispatch), in dispatch order, optionally only for kernels matching a regex."""
    vals = defaultdict(float)
    names = {}
    rx = re.compile(kernel_re) if kernel_re else None
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            if rx and not rx.search(r["Kernel_Name"]):
                continue
            d = int(r["Dispatch_Id"])
            vals[d] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
    order = sorted(vals)
    return [vals[d] for d in order], [names[d] for d in order]


def cmd_traffic(args):
    cf, _ = counter_values(args.calib_fetch, "FETCH_SIZE")
    cw, _ = counter_values(args.calib_write, "WRITE_SIZE")
    if not cf or not cw:
        sys.exit("no copy dispatches in the calibration runs")
    fetch_scale = COPY_BYTES / (statistics.median(cf) * 1024.0)
    write_scale = COPY_BYTES / (statistics.median(cw) * 1024.0)
    f, names = counter_values(args.fetch, "FETCH_SIZE", args.kernel_regex)
    w, _ = counter_values(args.write, "WRITE_SIZE", args.kernel_regex)
    if len(f) < args.last or len(w) < args.last:
        sys.exit(f"fewer than {args.last} matching dispatches ({len(f)}, {len(w)})")
    fb = statistics.mean(f[-args.last:]) * 1024.0 * fetch_scale
    wb = statistics.mean(w[-args.last:]) * 1024.0 * write_scale
    out = {}
    if os.path.exists(args.out):
        with open(args.out) as fh:
            out = json.load(fh)
    sha = kernel_sources_sha()
    if out.get("csrc_sha") != sha:
        out = {}
    out.update({"csrc_sha": sha, "fetch_scale": fetch_scale, "write_scale": write_scale,
                "calibration": f"device copy of {COPY_BYTES} bytes: FETCH_SIZE {statistics.median(cf):.0f} KiB, "
                               f"WRITE_SIZE {statistics.median(cw):.0f} KiB per dispatch"})
    out.setdefault("kernels", {})[args.family] = {
        "kernel": names[-1], "launches": args.last, "fetch_bytes": fb, "write_bytes": wb,
        "traffic_bytes": fb + wb, "algorithmic_bytes": args.algorithmic,
        "traffic_over_algorithmic": (fb + wb) / args.algorithmic if args.algorithmic else None,
        "command": args.command}
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"{args.family}: read {fb / 1e6:.1f} MB + write {wb / 1e6:.1f} MB per launch "
          f"(algorithmic {args.algorithmic / 1e6:.1f} MB); scales {fetch_scale:.3f} / {write_scale:.3f}")
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("window")
    a.add_argument("trace")
    a.add_argument("window")
    a.add_argument("--leg", default="headline")
    a.add_argument("--top", type=int, default=25)
    t = sub.add_parser("traffic")
    for k in ("--fetch", "--write", "--calib-fetch", "--calib-write", "--family", "--out"):
        t.add_argument(k, required=True)
    t.add_argument("--kernel-regex", required=True)
    t.add_argument("--last", type=int, default=200)
    t.add_argument("--algorithmic", type=float, default=0.0)
    t.add_argument("--command", default="")
    args = ap.parse_args(argv)
    return cmd_window(args) if args.cmd == "window" else cmd_traffic(args)


if __name__ == "__main__":
    sys.exit(main())

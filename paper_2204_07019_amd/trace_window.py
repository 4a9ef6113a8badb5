"""Kernel statistics of a rocprofv3 kernel trace inside a timed window.

rocprofv3 --kernel-trace --output-format csv writes one row per dispatch with
start and end timestamps.  bench.py --trace-window FILE records, for each timed
run, the host clocks (CLOCK_MONOTONIC and CLOCK_BOOTTIME, ns) at the
synchronised start and end of its timed steps.  This module keeps the
dispatches that start inside one such window and groups them by kernel name and
launch grid (the levels of a hierarchy share a name and differ in grid).

Within a group, launches that end after less than a fifth of the group's 90th
percentile duration are counted apart as short launches: the iterations of a
captured Krylov chunk that begin after convergence return at once, and a
level's first touch of cold data takes longer; the averages over the remaining
launches are the per-launch figures a roofline may use.

    python -m paper_2204_07019_amd.trace_window TRACE.csv WINDOW.json [--leg NAME] [--top N]
"""
from __future__ import annotations

import argparse
import csv
import json
import sys
from collections import defaultdict

SHORT_FRAC = 0.2


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
    """The host clock whose window holds dispatches (the one the trace's
    timestamps follow): the clock with the most dispatches starting inside."""
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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("trace")
    ap.add_argument("window")
    ap.add_argument("--leg", default="headline")
    ap.add_argument("--top", type=int, default=25)
    args = ap.parse_args(argv)
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
          f"kernel busy {total * 1e-6:.1f} ms ({total * 1e-9 / wall * 100:.1f} % of the window)\n")
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


if __name__ == "__main__":
    sys.exit(main())

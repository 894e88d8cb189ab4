"""Summaries of rocprofv3 output for the committed profiles.

    # per-kernel durations from --kernel-trace --stats (csv output)
    python -m paper_2609_22608_amd.prof_summary durations DIR --title "..." --command "..."

    # HBM traffic of one kernel (or of the kernels of one timed span, summed)
    # from two --pmc runs (FETCH_SIZE, WRITE_SIZE), calibrated by the 256 MiB
    # device copy that `bench.py --profile` runs
    python -m paper_2609_22608_amd.prof_summary traffic FETCH_DIR WRITE_DIR \\
        --kernel "edge_triage_kernel<5720, 1>" --kernel "tri_hist_kernel" ... \\
        --key edge_search --form screen/3 --command "..." --json profiles/traffic.json
    python -m paper_2609_22608_amd.prof_summary traffic FETCH_DIR WRITE_DIR \\
        --kernel "knn_scan<12, 4>" --key knn_scan --form 1 --json profiles/traffic.json

Durations are per dispatch (End - Start of the kernel trace).  Traffic:
FETCH_SIZE and WRITE_SIZE are KiB per dispatch; each is divided by what the
same counter reads for the plain copy of known size (bytes moved each way),
so the result is bytes per launch.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import statistics
import sys

COPY_BYTES = 256 << 20  # the calibration copy of bench.py --profile
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _one(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def short(name, width=64):
    name = name.replace("void ", "").replace("fn::", "")
    p = name.find("(")
    if p > 0:
        name = name[:p]
    return name if len(name) <= width else name[: width - 3] + "..."


def durations(args):
    rows = list(csv.DictReader(open(_one(args.dir, "kernel_trace.csv"))))
    per = collections.defaultdict(list)
    for r in rows:
        per[short(r["Kernel_Name"])].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in per.values())
    out = [f"# {args.title}", "", "Command (from the repository root):", "", "```", args.command,
           "```", "", "| kernel | calls | mean us | median us | min us | max us | share |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) / total < args.min_share:
            continue
        out.append(f"| `{k}` | {len(v)} | {statistics.mean(v):.1f} | {statistics.median(v):.1f} | "
                   f"{min(v):.1f} | {max(v):.1f} | {100 * sum(v) / total:.1f}% |")
    print("\n".join(out))


def _counter(d, name, grid=None):
    """{kernel: [value per dispatch]} (dispatches of grid size `grid` only,
    when given), {(kernel, grid): [value per dispatch]} and the copy
    calibration value."""
    rows = list(csv.DictReader(open(_one(d, "counter_collection.csv"))))
    per = collections.defaultdict(list)
    per_grid = collections.defaultdict(list)
    copy = []
    for r in rows:
        if r["Counter_Name"] != name:
            continue
        v = float(r["Counter_Value"])
        g = int(r["Grid_Size"])
        if r["Kernel_Name"] == COPY_KERNEL:
            copy.append((g, v))
        per_grid[(short(r["Kernel_Name"], 200), g)].append(v)
        if grid is None or g == grid:
            per[short(r["Kernel_Name"], 200)].append(v)
    if not copy:
        raise SystemExit(f"no {COPY_KERNEL} dispatch in {d}")
    grid, cal = max(copy)  # the large calibration copy
    return per, per_grid, cal, grid


def traffic(args):
    fetch, fetch_g, f_cal, grid = _counter(args.fetch, "FETCH_SIZE", args.grid)
    write, write_g, w_cal, _ = _counter(args.write, "WRITE_SIZE", args.grid)
    kib = COPY_BYTES / 1024
    f_scale = f_cal / kib  # counter KiB per KiB moved
    w_scale = w_cal / kib
    print(f"calibration copy (grid {grid}): FETCH_SIZE {f_cal:.0f} KiB, WRITE_SIZE {w_cal:.0f} KiB "
          f"for {kib:.0f} KiB moved each way -> scale 1/{f_scale:.3f}, 1/{w_scale:.3f}")
    # the kernels of one timed span each run once per span: their means add
    fk = wk = 0.0
    counts = []
    for kname in args.kernel:
        # "name@grid": only that kernel's dispatches of that grid size
        g = None
        if "@" in kname:
            kname, g = kname.rsplit("@", 1)
            g = int(g)
        key = short(kname, 200)
        fl = fetch.get(key) if g is None else fetch_g.get((key, g))
        wl = write.get(key) if g is None else write_g.get((key, g))
        if not fl or not wl:
            raise SystemExit(f"{key} (grid {g}) not found; kernels: {sorted(fetch)}")
        f1, w1 = statistics.mean(fl), statistics.mean(wl)
        print(f"{key}{'' if g is None else f' (grid {g})'}: FETCH_SIZE {f1:.0f} KiB, WRITE_SIZE "
              f"{w1:.0f} KiB per dispatch ({len(fl)}, {len(wl)} dispatches)")
        fk += f1
        wk += w1
        counts.append([len(fl), len(wl)])
    fb = fk / f_scale * 1024
    wb = wk / w_scale * 1024
    print(f"per launch: {fb / 1e6:.3f} MB read + {wb / 1e6:.3f} MB written = "
          f"{(fb + wb) / 1e6:.3f} MB")
    if args.json:
        sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        from bench import kernel_source_hash

        base = args.key or args.kernel[0].split("<")[0]
        data = {}
        if os.path.exists(args.json):
            data = json.load(open(args.json))
        data[base] = dict(kernel=" + ".join(args.kernel), form=args.form,
                          source_hash=kernel_source_hash(base), fetch_kib=fk, write_kib=wk,
                          fetch_scale=f_scale, write_scale=w_scale, bytes_per_launch=fb + wb,
                          command=args.command,
                          dispatches=counts[0] if len(counts) == 1 else counts, grid=args.grid)
        with open(args.json, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    d = sub.add_parser("durations")
    d.add_argument("dir")
    d.add_argument("--title", default="Kernel durations")
    d.add_argument("--command", default="")
    d.add_argument("--min-share", type=float, default=0.001)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("--kernel", required=True, action="append",
                   help="kernel name, or name@grid for that grid size's dispatches only; "
                        "repeated: the kernels of one timed span, summed")
    t.add_argument("--form", required=True)
    t.add_argument("--grid", type=int, default=None,
                   help="only dispatches of this grid size (work-items), e.g. the tuned mapping")
    t.add_argument("--key", default=None,
                   help="record name (default: the kernel name without template arguments)")
    t.add_argument("--command", default="")
    t.add_argument("--json", default=None)
    a = ap.parse_args()
    durations(a) if a.cmd == "durations" else traffic(a)


if __name__ == "__main__":
    main()

"""Summaries of rocprofv3 output for the measurement records.

- `stats` turns a `--kernel-trace --stats` run's kernel_stats.csv into a short Markdown table.
- `traffic` turns two `--pmc` runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) into bytes per
  launch of the solve kernels. The counters are scaled by what they read for a calibration kernel
  of known traffic in the same run: an elementwise negation of a float64 buffer of known size,
  which reads and writes that size once.

python -m paper_2406_00991_amd.profiling stats <kernel_stats.csv> --command "<cmd>" > out.md
python -m paper_2406_00991_amd.profiling traffic <fetch dir> <write dir> --copy-bytes B \
       --command "<cmd>" > out.json
"""
import argparse
import csv
import glob
import json
import os
import re
import sys


def _find(root, name):
    hits = sorted(glob.glob(os.path.join(root, "**", name), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {name} under {root}")
    return hits


def stats(csv_path, command, top=12):
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"Command: `{command}`", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"].split("(")[0]
        out.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _per_kernel(root, counter):
    """{kernel name: [value per dispatch]} of one counter from counter_collection.csv files."""
    vals = {}
    for path in _find(root, "*counter_collection.csv"):
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_dir, write_dir, copy_bytes, command, source_sha256, prefix="k_solve"):
    fetch = _per_kernel(fetch_dir, "FETCH_SIZE")
    write = _per_kernel(write_dir, "WRITE_SIZE")
    cal = [k for k in fetch if "neg" in k.lower()]
    if not cal:
        raise RuntimeError("calibration kernel (negation) not found in the FETCH_SIZE run")
    calw = [k for k in write if "neg" in k.lower()]
    # the calibration kernel reads copy_bytes and writes copy_bytes
    f_cal = max(max(fetch[k]) for k in cal) * 1024.0
    w_cal = max(max(write[k]) for k in calw) * 1024.0
    ffac, wfac = copy_bytes / f_cal, copy_bytes / w_cal
    rec = {"command": command, "source_sha256": source_sha256,
           "calibration": {"bytes": copy_bytes, "fetch_read": f_cal, "write_read": w_cal,
                           "fetch_factor": ffac, "write_factor": wfac},
           "kernels": {}}
    for k, v in fetch.items():
        m = re.search(r"pmgw::(\w+)<(float|double), (\d+)(?:, \d+, (true|false)"
                      r"(?:, (true|false))?)?", k)
        if not m or not m.group(1).startswith(prefix) or m.group(4) == "true":
            continue
        w = write.get(k, [0.0])
        fb = ffac * 1024.0 * sum(v) / len(v)
        wb = wfac * 1024.0 * sum(w) / len(w)
        prec = "mixed" if m.group(2) == "float" else "fp64"
        res = ",res" if m.group(5) == "true" else ""
        key = f"{m.group(1)}<{m.group(2)},{m.group(3)}{res}>/{prec}"
        rec["kernels"][key] = {"dispatches": len(v), "fetch_bytes": fb, "write_bytes": wb,
                               "bytes_per_launch": fb + wb}
    return rec


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--top", type=int, default=12, help="rows of the table (kernels by total time)")
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--source-sha256", required=True)
    args = ap.parse_args()
    if args.cmd == "stats":
        sys.stdout.write(stats(args.csv, args.command, args.top))
    else:
        json.dump(traffic(args.fetch_dir, args.write_dir, args.copy_bytes, args.command,
                          args.source_sha256), sys.stdout, indent=1)
        sys.stdout.write("\n")


if __name__ == "__main__":
    main()

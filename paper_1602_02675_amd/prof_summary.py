"""Summarise rocprofv3 output of `bench.py --profile` into profiles/.

Reads a kernel-trace `--stats` directory and two counter directories
(FETCH_SIZE, WRITE_SIZE; one pass each), and writes
  profiles/<name>.txt   the figures used, with the commands that made them
  profiles/traffic_<name>.json  HBM bytes per step-kernel launch, with the
                        source hash of the kernel it was measured on.
HBM bytes = counter KiB * 1024 / (counter KiB * 1024 per byte of a plain
device copy of 1 GiB run in the same process), per dispatch, averaged.

Usage (after the three rocprofv3 runs):
  python -m paper_1602_02675_amd.prof_summary --stats DIR --fetch DIR --write DIR \
      --name march2d_fp64_4096 --kernel march2d_kernel --cmd "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30


def _csvs(d, pattern):
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def kernel_stats(d):
    rows = []
    for f in _csvs(d, "*kernel_stats.csv"):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def counter_values(d, counter):
    """{kernel name: [per-dispatch value]} for one counter."""
    out = {}
    for f in _csvs(d, "*counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _pick(d, sub):
    keys = [k for k in d if sub in k]
    if not keys:
        raise SystemExit(f"no kernel matching {sub!r}; have: {list(d)[:20]}")
    vals = []
    for k in keys:
        vals += d[k]
    return keys, vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--name", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--copy-kernel", default="copyBuffer")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--bytes-per-launch", type=float, required=True,
                    help="algorithmic bytes per step-kernel launch")
    ap.add_argument("--sources", nargs="*", default=None,
                    help="kernel source files whose hash is recorded (default: the benchmark's step kernel)")
    args = ap.parse_args()

    sys.path.insert(0, ROOT)
    import bench

    stats = kernel_stats(args.stats)
    krow = [r for r in stats if args.kernel in r.get("Name", "")]
    if not krow:
        raise SystemExit("kernel not in stats")
    kr = krow[0]
    avg_ns = float(kr["AverageNs"])
    fetch = counter_values(args.fetch, "FETCH_SIZE")
    write = counter_values(args.write, "WRITE_SIZE")
    _, kf = _pick(fetch, args.kernel)
    _, kw = _pick(write, args.kernel)
    _, cf = _pick(fetch, args.copy_kernel)
    _, cw = _pick(write, args.copy_kernel)
    # the calibration copies are the three largest copy dispatches (1 GiB
    # each); smaller copies of the run (staging, exports) are not used
    cf, cw = sorted(cf)[-3:], sorted(cw)[-3:]
    f_factor = (sum(cf) / len(cf)) * 1024.0 / COPY_BYTES
    w_factor = (sum(cw) / len(cw)) * 1024.0 / COPY_BYTES
    fetch_b = (sum(kf) / len(kf)) * 1024.0 / f_factor
    write_b = (sum(kw) / len(kw)) * 1024.0 / w_factor
    traffic = fetch_b + write_b
    res = {
        "kernel": kr["Name"],
        "kernel_source_sha": bench.kernel_source_sha(args.sources),
        "calls": int(kr["Calls"]),
        "avg_duration_us": avg_ns / 1e3,
        "fetch_kib_per_launch": sum(kf) / len(kf),
        "write_kib_per_launch": sum(kw) / len(kw),
        "copy_fetch_factor": f_factor,
        "copy_write_factor": w_factor,
        "hbm_bytes_per_launch": traffic,
        "algorithmic_bytes_per_launch": args.bytes_per_launch,
        "traffic_over_algorithmic": traffic / args.bytes_per_launch,
        "achieved_GBs_from_trace": args.bytes_per_launch / (avg_ns * 1e-9) / 1e9,
    }
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"traffic_{args.name}.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    lines = [f"# {args.name}: rocprofv3 summary", "", f"command: {args.cmd}", "",
             "kernel-trace --stats (top kernels):"]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0)))[:8]:
        lines.append(f"  {r['Name'][:90]:90s} calls={r['Calls']:>6s} avg_us={float(r['AverageNs'])/1e3:10.2f}"
                     f" total_ms={float(r['TotalDurationNs'])/1e6:10.3f}")
    lines += ["", "counters (per dispatch of the step kernel):"]
    lines += [f"  {k}: {v}" for k, v in res.items()]
    with open(os.path.join(ROOT, "profiles", f"{args.name}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(res))


if __name__ == "__main__":
    main()

"""Summarise rocprofv3 output of `bench.py --profile` into profiles/.

Reads a kernel-trace `--stats` directory, two counter directories
(FETCH_SIZE, WRITE_SIZE; one pass each) and optionally further counter
directories (SQ instruction and cycle counters, one pass each), all written
with `--output-format csv`, and writes
  profiles/<name>.txt   the figures used, with the commands that made them
  profiles/traffic_<name>.json  HBM bytes per step, with the source hash of
                        the kernels it was measured on.
A step may be several kernels (the square lattice's lean, short and full
passes): every kernel whose name contains --kernel counts, and the per-step
figures are the sums of the per-kernel averages per dispatch.
HBM bytes = counter KiB * 1024 / (counter KiB * 1024 per byte of a plain
device copy of 1 GiB run in the same process).

Usage (after the rocprofv3 runs):
  python -m paper_1602_02675_amd.prof_summary --stats DIR --fetch DIR --write DIR [--counters DIR ...] \
      --name march2d_fp64_4096 --kernel march2d --bytes-per-launch N --cmd "..."
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


def kernel_resources(d, sub):
    """{kernel name: (VGPRs, AGPRs, SGPRs, LDS bytes, scratch bytes)} from the kernel trace."""
    out = {}
    for f in _csvs(d, "*kernel_trace.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                name = r.get("Kernel_Name", "")
                if sub in name and name not in out:
                    out[name] = tuple(r.get(k, "?") for k in ("VGPR_Count", "Accum_VGPR_Count", "SGPR_Count",
                                                               "LDS_Block_Size", "Scratch_Size"))
    return out


def counter_values(d, counter=None):
    """{(kernel name, counter): [per-dispatch value]} (one counter, or all)."""
    out = {}
    for f in _csvs(d, "*counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if counter is not None and r.get("Counter_Name") != counter:
                    continue
                out.setdefault((r["Kernel_Name"], r["Counter_Name"]), []).append(float(r["Counter_Value"]))
    return out


def per_step(vals, sub, counter):
    """Sum over the kernels matching `sub` of their average per dispatch."""
    keys = [k for k in vals if sub in k[0] and k[1] == counter]
    if not keys:
        raise SystemExit(f"no kernel matching {sub!r} with {counter}; have: {sorted(set(k[0] for k in vals))[:20]}")
    return sum(sum(vals[k]) / len(vals[k]) for k in keys), keys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--counters", nargs="*", default=[], help="further counter directories (SQ_*, GRBM_*)")
    ap.add_argument("--name", required=True)
    ap.add_argument("--kernel", required=True, help="substring naming the step's kernels")
    ap.add_argument("--copy-kernel", default="copyBuffer")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--clock-ghz", type=float, default=2.4)
    ap.add_argument("--cus", type=int, default=256)
    ap.add_argument("--bytes-per-launch", type=float, required=True,
                    help="algorithmic bytes per step")
    ap.add_argument("--sources", nargs="*", default=None,
                    help="kernel source files whose hash is recorded (default: the benchmark's step kernel)")
    args = ap.parse_args()

    sys.path.insert(0, ROOT)
    import bench

    stats = kernel_stats(args.stats)
    krows = [r for r in stats if args.kernel in r.get("Name", "")]
    if not krows:
        raise SystemExit("kernel not in stats")
    step_ns = sum(float(r["AverageNs"]) for r in krows)
    fetch = counter_values(args.fetch, "FETCH_SIZE")
    write = counter_values(args.write, "WRITE_SIZE")
    kf, _ = per_step(fetch, args.kernel, "FETCH_SIZE")
    kw, _ = per_step(write, args.kernel, "WRITE_SIZE")
    # the calibration copies are the three largest copy dispatches (1 GiB
    # each); smaller copies of the run (staging, exports) are not used
    cf = sorted(v for (k, c), vs in fetch.items() if args.copy_kernel in k for v in vs)[-3:]
    cw = sorted(v for (k, c), vs in write.items() if args.copy_kernel in k for v in vs)[-3:]
    f_factor = (sum(cf) / len(cf)) * 1024.0 / COPY_BYTES
    w_factor = (sum(cw) / len(cw)) * 1024.0 / COPY_BYTES
    fetch_b = kf * 1024.0 / f_factor
    write_b = kw * 1024.0 / w_factor
    traffic = fetch_b + write_b
    res = {
        "kernels": [r["Name"] for r in krows],
        "kernel_source_sha": bench.kernel_source_sha(args.sources),
        "calls": [int(r["Calls"]) for r in krows],
        "avg_duration_us": [float(r["AverageNs"]) / 1e3 for r in krows],
        "step_duration_us": step_ns / 1e3,
        "fetch_kib_per_step": kf,
        "write_kib_per_step": kw,
        "copy_fetch_factor": f_factor,
        "copy_write_factor": w_factor,
        "hbm_bytes_per_launch": traffic,
        "algorithmic_bytes_per_launch": args.bytes_per_launch,
        "traffic_over_algorithmic": traffic / args.bytes_per_launch,
        "achieved_GBs_from_trace": args.bytes_per_launch / (step_ns * 1e-9) / 1e9,
    }
    # SQ counters of the dominant kernel (the longest of the step)
    dom = max(krows, key=lambda r: float(r["AverageNs"]))["Name"]
    sq = {}
    for d in args.counters:
        for (k, c), vs in counter_values(d).items():
            if k == dom:
                sq[c] = sum(vs) / len(vs)
    derived = {}
    if sq:
        dom_ns = float(next(r["AverageNs"] for r in krows if r["Name"] == dom))
        # the kernel's own duration in shader-clock cycles (GRBM_GUI_ACTIVE
        # is summed over the chip's 8 XCDs, and spans more than the kernel)
        cycles = dom_ns * 1e-9 * args.clock_ghz * 1e9
        simds = 4 * args.cus
        if "SQ_ACTIVE_INST_VALU" in sq:  # quad-cycles per SE aggregate over SIMDs
            derived["valu_busy"] = 4.0 * sq["SQ_ACTIVE_INST_VALU"] / simds / cycles
        waves = sq.get("SQ_WAVES")
        if waves:
            for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_BRANCH", "SQ_INSTS_VALU_FMA_F64",
                      "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64"):
                if c in sq:
                    derived[c.lower().replace("sq_insts_", "per_wave_")] = sq[c] / waves
        if "SQ_WAVE_CYCLES" in sq:
            for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY"):
                if c in sq:
                    derived[c.lower() + "_frac_of_wave_cycles"] = sq[c] / sq["SQ_WAVE_CYCLES"]
    res["dominant_kernel"] = dom
    res["dominant_counters"] = sq
    res["dominant_derived"] = derived
    res["resources"] = {k: dict(zip(("vgpr", "agpr", "sgpr", "lds_bytes", "scratch_bytes"), v))
                        for k, v in kernel_resources(args.stats, args.kernel).items()}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"traffic_{args.name}.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    lines = [f"# {args.name}: rocprofv3 summary", "", f"command: {args.cmd}", "",
             "kernel-trace --stats (top kernels):"]
    for r in sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0)))[:8]:
        lines.append(f"  {r['Name'][:90]:90s} calls={r['Calls']:>6s} avg_us={float(r['AverageNs'])/1e3:10.2f}"
                     f" total_ms={float(r['TotalDurationNs'])/1e6:10.3f}")
    lines += ["", "kernel resources (kernel trace): VGPRs, AGPRs, SGPRs, LDS bytes, scratch bytes per lane"]
    lines += [f"  {k[:90]}: {v}" for k, v in res["resources"].items()]
    lines += ["", "per step (sum over the step's kernels):"]
    lines += [f"  {k}: {v}" for k, v in res.items() if k not in ("resources", "dominant_counters", "dominant_derived")]
    if sq:
        lines += ["", f"counters of the dominant kernel (per dispatch): {dom[:90]}"]
        lines += [f"  {k}: {v:.6g}" for k, v in sorted(sq.items())]
        lines += ["", "derived (valu_busy: VALU issue quad-cycles / (SIMDs x cycles); per_wave_*: instructions per wavefront)"]
        lines += [f"  {k}: {v:.4g}" for k, v in derived.items()]
    with open(os.path.join(ROOT, "profiles", f"{args.name}.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({k: v for k, v in res.items() if k != "resources"}))


if __name__ == "__main__":
    main()

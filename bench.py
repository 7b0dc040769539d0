#!/usr/bin/env python3
"""Benchmark of the tau = 1 semi-discrete LB step on one MI355X.

Workload: a 2-D planar shock tube on the square dual-level lattice,
4096 x 4096 nodes, seeded Riemann state (rho_L = 1, p_L = 1, u = 0; pressure
ratio log-uniform in [2, 100], density ratio in [1, 10], diaphragm in
[0.3, 0.7]; seed 0), lambda from the CFL bound of the initial states,
transmissive in x, periodic in y.  A step is one pass of the whole step (the
fused gather kernel plus its totals reduction).  The FP64 plain form is the
headline number; the FP32 form runs the same workload for comparison
(node-updates/s and relative L1 density error against FP64).

Prints one JSON line.  `--profile` runs a short version plus a plain device
copy of known size, for rocprofv3 counter runs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-updates/s (MLUPS) + % HBM peak; FP32-batched vs FP64 plain at L1<=1e-5"
HBM_PEAK_GBS = 8000.0
NX = NY = 4096
SEED = 0
BYTES_PER_NODE = {"fp64": 64, "fp32": 32}  # read 4 moment fields + write 4 (algorithmic)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_march2d_fp64_4096.json")
KERNEL_SOURCES = ["paper_1602_02675_amd/csrc/lb_march2d.hip", "paper_1602_02675_amd/csrc/lb_device.hpp"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload():
    from paper_1602_02675_amd import inputs

    left, right, x_d = inputs.riemann_instance(SEED)
    lam = inputs.cfl_lambda([left, right])
    return left, right, x_d, lam


def run_gpu(precision: str, steps: int, warmup: int):
    import torch
    from paper_1602_02675_amd.lbsd import Solver

    left, right, x_d, lam = workload()
    s = Solver(2, NX, NY, precision=precision, bc_x="transmissive", bc_y="periodic")
    s.init_riemann(x_d, left, right, lam=lam)
    if warmup:
        s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kernel_ms, total_ms = s.step_profiled(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rho = s.moments_device()[0].clone()
    s.close()
    return dict(kernel_ms=kernel_ms, total_ms=total_ms, wall_s=wall, rho=rho)


def cpu_baseline(seconds_target: float = 15.0):
    """The oracle, single-threaded, on a bounded sample of the same workload."""
    import oracle
    from paper_1602_02675_amd import inputs

    left, right, x_d, lam = workload()
    n = 512
    P = oracle.Problem(2, n, n)
    Y = oracle.to_lattice(P, oracle.riemann_moments(P, inputs.node_x(n), left, right, x_d), lam)
    steps = 2
    t0 = time.perf_counter()
    Y, st, _ = oracle.run(P, Y, steps)
    dt = time.perf_counter() - t0
    more = max(1, int(seconds_target / max(dt / steps, 1e-6)) - steps)
    more = min(more, 200)
    t0 = time.perf_counter()
    Y, st, _ = oracle.run(P, Y, more)
    dt = time.perf_counter() - t0
    return dict(value=n * n * more / dt / 1e6, unit="MLUPS", cores=1, kind="oracle",
                sample=f"{n}x{n} nodes of the same seeded planar tube, {more} steps, FP64, 1 thread")


def traffic_per_launch():
    """HBM bytes per step-kernel launch from the committed counter summary,
    or None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short run + a plain copy of known size, for rocprofv3 counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.profile:
        # plain device copy of 1 GiB, three times (counter calibration)
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        r = run_gpu("fp64", args.steps, args.warmup)
        print(json.dumps({"profile": True, "steps": args.steps, "kernel_ms": r["kernel_ms"],
                          "kernel_source_sha": kernel_source_sha()}), flush=True)
        return

    nodes = NX * NY
    r64 = run_gpu("fp64", args.steps, args.warmup)
    total_s = r64["total_ms"] / 1e3
    mlups = nodes * args.steps / total_s / 1e6
    kernel_s_per_launch = r64["kernel_ms"] / 1e3 / args.steps
    achieved = BYTES_PER_NODE["fp64"] * nodes / kernel_s_per_launch / 1e9
    traffic = traffic_per_launch()
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["total_ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2-D planar shock tube, square dual-level lattice, 4096x4096 nodes, "
                               "seeded Riemann state (seed 0), CFL 1, transmissive x / periodic y",
                   "nx": NX, "ny": NY, "seed": SEED, "precision": "fp64", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "march2d_kernel<double>",
                     "kernel_us_per_launch": round(kernel_s_per_launch * 1e6, 2),
                     "algorithmic_bytes_per_launch": BYTES_PER_NODE["fp64"] * nodes},
    }
    if not args.no_fp32:
        r32 = run_gpu("fp32", args.steps, args.warmup)
        rho64, rho32 = r64["rho"], r32["rho"]
        rel_l1 = float((rho32 - rho64).abs().sum() / rho64.abs().sum())
        out["fp32"] = {"value": round(nodes * args.steps / (r32["total_ms"] / 1e3) / 1e6, 1), "unit": "MLUPS",
                       "ms_per_step": round(r32["total_ms"] / args.steps, 5),
                       "rel_l1_density_vs_fp64": rel_l1,
                       "achieved_GBs": round(BYTES_PER_NODE["fp32"] * nodes /
                                             (r32["kernel_ms"] / 1e3 / args.steps) / 1e9, 1)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

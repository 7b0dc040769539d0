#!/usr/bin/env python3
"""Benchmark of the tau = 1 semi-discrete LB step on one MI355X.

Headline: a 2-D planar shock tube on the square dual-level lattice,
4096 x 4096 nodes, seeded Riemann state (rho_L = 1, p_L = 1, u = 0; pressure
ratio log-uniform in [2, 100], density ratio in [1, 10], diaphragm in
[0.3, 0.7]; seed 0), lambda from the CFL bound of the initial states,
transmissive in x, periodic in y; FP64 plain form, one step = the fused
gather kernel plus its totals reduction.  Alongside, in the same JSON line:

* fp32:  the same workload in the FP32 form (node-updates/s and relative L1
  density error against FP64 after the timed steps);
* batch: 512 independent 1-D tubes, lengths log-uniform in [256, 65536],
  seeded states, 1000 steps, one persistent launch per step over all tubes,
  HIP-graph captured, tile shape autotuned, FP32 and FP64;
* walls: the headline tube between reflecting walls at both x ends (FP64;
  the kernel instances that handle walls);
* nonplanar: a seeded four-state 2-D Riemann problem (both velocity
  components of both signs) on 2048 x 2048 nodes, FP64;
* hex: the headline tube on the hexagonal lattice (4096 x 4096 nodes, state
  along the axial index i), FP64, 100 steps;
* rest_level: the headline tube on the square lattice with a rest level
  (d_0 = rho / 2), FP64, 100 steps;
* tube1d / tube1d_fp32 / two_gas: one 1-D Sod tube of 2^24 nodes, 200
  steps: FP64 and FP32 with one gas, FP64 with gamma 7/5 | 5/3 on the two
  sides (species field);
* two_gas2d: the headline tube with gamma 5/3 on the right (species field
  on the square lattice), FP64, 100 steps;
* batch2d: 48 planar square-lattice tubes of uneven sizes (nx log-uniform in
  [256, 4096], ny in [64, 1024]), seeded states, one pool, autotuned tiles,
  HIP-graph steps, 250 steps, FP32 and FP64 (and the FP32 density error
  against FP64);
* serve: square-lattice requests (sides log-uniform in [64, 2048], steps in
  [100, 5000], seeded states) arriving as a Poisson process at 0.5, 0.8 and
  1.0 x the measured capacity, continuously batched on an FP32 pool: p50 /
  p99 latency and served node-updates/s at each load (the headline figures
  at 0.8); and the same requests all queued at once (the served throughput
  at saturation);
* cpu_baseline: the FP64 oracle on a bounded sample, one host thread (host
  CPU model and usable cores stated); cpu_baseline_batch: the oracle over the
  512 independent tubes of the batch workload on all usable cores (at most
  16), one process per core.
* fp32.rel_l1_density_vs_fp64_2000_steps: the FP32 form's density error
  against FP64 after the 2000 steps the FP32-versus-FP64 comparison is
  stated at (a 4096 x 16 strip of the headline tube: planar rows evolve
  bit-identically), whatever --steps is; and the same for the tubes of
  seeds 0-7 of the family.

`--profile` runs a short headline plus a plain device copy of known size,
for rocprofv3 counter runs (`--profile-batch`, `--profile-hex`: the same for
the FP64 tube batch and the hexagonal-lattice tube).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-updates/s (MLUPS) + % HBM peak; FP32-batched vs FP64 plain at L1<=1e-5"
HBM_PEAK_GBS = 8000.0
NX = NY = 4096
SEED = 0
BYTES_PER_NODE = {"fp64": 64, "fp32": 32}  # read 4 moment fields + write 4 (algorithmic)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_march2d_fp64_4096.json")
KERNEL_SOURCES = ["paper_1602_02675_amd/csrc/lb_march2d.hpp", "paper_1602_02675_amd/csrc/lb_march2d.hip",
                  "paper_1602_02675_amd/csrc/lb_device.hpp", "paper_1602_02675_amd/csrc/lb_kernels.hpp"]


def kernel_source_sha(sources=None) -> str:
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload(seed: int = SEED):
    from paper_1602_02675_amd import inputs

    left, right, x_d = inputs.riemann_instance(seed)
    lam = inputs.cfl_lambda([left, right])
    return left, right, x_d, lam


def run_gpu(precision: str, steps: int, warmup: int, bc_x: str = "transmissive", d0_frac: float = 0.0,
            gamma2=None):
    """The headline tube; with gamma2, gas 2 on the right (lambda then from
    CFL 1 over both sides, each with its own gamma)."""
    import torch
    from paper_1602_02675_amd.lbsd import Solver

    left, right, x_d, lam = workload()
    s = Solver(2, NX, NY, precision=precision, bc_x=bc_x, bc_y="periodic", d0_frac=d0_frac, gamma2=gamma2)
    s.init_riemann(x_d, left, right, lam=None if gamma2 else lam)
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


def run_nonplanar(steps: int = 200, n: int = 2048, seed: int = 1):
    """Four-state 2-D Riemann problem (non-planar data), FP64, transmissive."""
    import torch
    from paper_1602_02675_amd import inputs
    from paper_1602_02675_amd.lbsd import Solver

    states, center = inputs.quadrant_riemann(seed)
    lam = inputs.quadrant_lambda(states)
    s = Solver(2, n, n, precision="fp64", bc_x="transmissive", bc_y="transmissive")
    s.init_moments(inputs.quadrant_moments(states, center, n, n), lam)
    s.step(10)
    s.sync()
    torch.cuda.synchronize()
    kernel_ms, total_ms = s.step_profiled(steps)
    s.close()
    return dict(value=round(n * n * steps / (total_ms * 1e-3) / 1e6, 1), unit="MLUPS", nx=n, ny=n, seed=seed,
                steps=steps, ms_per_step=round(total_ms / steps, 5), precision="fp64")


def run_hex(steps: int = 100, precision: str = "fp64"):
    """The headline tube on the hexagonal lattice (nodes at i e_1 + j e_2;
    the state depends on the axial index i, transmissive along i, periodic
    along j), 4096 x 4096."""
    import torch
    from paper_1602_02675_amd.lbsd import Solver

    left, right, x_d, lam = workload()
    s = Solver(2, NX, NY, precision=precision, bc_x="transmissive", bc_y="periodic", lattice="hex")
    s.init_riemann(x_d, left, right, lam=lam)
    s.step(5)
    s.sync()
    torch.cuda.synchronize()
    kernel_ms, total_ms = s.step_profiled(steps)
    s.close()
    nodes = NX * NY
    return dict(value=round(nodes * steps / (total_ms * 1e-3) / 1e6, 1), unit="MLUPS", nx=NX, ny=NY, steps=steps,
                ms_per_step=round(total_ms / steps, 5),
                achieved_GBs=round(BYTES_PER_NODE[precision] * nodes / (kernel_ms * 1e-3 / steps) / 1e9, 1),
                precision=precision, lattice="hexagonal")


def run_tube1d(gamma2=None, n: int = 1 << 24, steps: int = 200, precision: str = "fp64"):
    """One long 1-D Sod tube; with gamma2, gas 2 on the right."""
    import torch
    from paper_1602_02675_amd import inputs
    from paper_1602_02675_amd.lbsd import Solver

    s = Solver(1, n, gamma=1.4, gamma2=gamma2, precision=precision)
    s.init_riemann(0.5, inputs.SOD_LEFT, inputs.SOD_RIGHT)
    s.step(5)
    s.sync()
    torch.cuda.synchronize()
    kernel_ms, total_ms = s.step_profiled(steps)
    s.close()
    nf = 3 if gamma2 is None else 4
    elem = 8 if precision == "fp64" else 4
    return dict(value=round(n * steps / (total_ms * 1e-3) / 1e6, 1), unit="MLUPS", nodes=n, steps=steps,
                ms_per_step=round(total_ms / steps, 5),
                achieved_GBs=round(2 * nf * elem * n / (kernel_ms * 1e-3 / steps) / 1e9, 1), precision=precision,
                gammas=[1.4] if gamma2 is None else [1.4, gamma2])


def host_info():
    """CPU model and the cores this process may use (a host may grant it a
    share of its cores, whatever os.cpu_count() reports)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable


def _oracle_tubes(job):
    """Worker of cpu_baseline_batch (a spawned process): the 1-D oracle on
    the given seeded tubes for `steps` steps; returns (node-updates, seconds)."""
    import oracle
    from paper_1602_02675_amd import inputs

    tubes, steps = job
    work, busy = 0, 0.0
    for L, i, seed in tubes:
        left, right, xd = inputs.riemann_instance(seed * 100000 + i)
        P = oracle.Problem(1, L)
        Y = oracle.to_lattice(P, oracle.riemann_moments(P, inputs.node_x(L), left, right, xd),
                              inputs.cfl_lambda([left, right]))
        t0 = time.perf_counter()
        oracle.run(P, Y, steps)
        busy += time.perf_counter() - t0
        work += L * steps
    return work, busy


def cpu_baseline_batch(seconds_target: float = 15.0, n_tubes: int = 512, seed: int = 0):
    """The oracle over the independent tubes of the batch workload (512 seeded
    1-D tubes, lengths log-uniform in [256, 65536]) on all usable host cores,
    one process per core, each taking whole tubes (balanced by length)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    from paper_1602_02675_amd import inputs

    model, usable = host_info()
    cores = max(1, min(16, usable))
    lens = [int(L) for L in inputs.tube_lengths(seed, n_tubes)]
    order = sorted(range(n_tubes), key=lambda i: -lens[i])
    shares = [[] for _ in range(cores)]
    load = [0] * cores
    for i in order:  # longest first onto the least loaded core
        c = load.index(min(load))
        shares[c].append((lens[i], i, seed))
        load[c] += lens[i]
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=cores, mp_context=ctx) as ex:
        # calibration: the workers start (and load the oracle) on a first
        # step of everything, a timed second pass of 2 steps sets the step
        # count for the target
        list(ex.map(_oracle_tubes, [(sh, 1) for sh in shares]))
        t0 = time.perf_counter()
        list(ex.map(_oracle_tubes, [(sh, 2) for sh in shares]))
        per_step = (time.perf_counter() - t0) / 2
        steps = int(min(1000, max(5, seconds_target / max(per_step, 1e-6))))
        t0 = time.perf_counter()
        res = list(ex.map(_oracle_tubes, [(sh, steps) for sh in shares]))
        wall = time.perf_counter() - t0
    work = sum(r[0] for r in res)
    return dict(value=work / wall / 1e6, unit="MLUPS", cores=cores, kind="oracle", host_cpu=model, nproc=usable,
                sample=f"all {n_tubes} tubes of the batch workload ({sum(lens)} nodes), {steps} steps, FP64, "
                       f"{cores} processes (whole tubes each, balanced by length)")


def fp32_accuracy(steps: int = 2000, ny: int = 16, seed: int = SEED):
    """Relative L1 density error of the FP32 form against FP64 on the headline
    tube (of the seeded family: `seed`) after `steps` steps, on a 4096 x ny
    periodic strip: a planar flow's rows evolve bit-identically, so every row
    of the 4096 x 4096 run is one of these rows."""
    import torch
    from paper_1602_02675_amd.lbsd import Solver

    left, right, x_d, lam = workload(seed)
    rho = {}
    for prec in ("fp64", "fp32"):
        s = Solver(2, NX, ny, precision=prec, bc_x="transmissive", bc_y="periodic")
        s.init_riemann(x_d, left, right, lam=lam)
        s.step(steps)
        y = s.moments()
        assert np.all(y == y[:, :1, :]), "planar rows differ"
        rho[prec] = y[0, 0]
        s.close()
    torch.cuda.synchronize()
    return float(np.sum(np.abs(rho["fp32"] - rho["fp64"])) / np.sum(np.abs(rho["fp64"])))


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
    model, usable = host_info()
    return dict(value=n * n * more / dt / 1e6, unit="MLUPS", cores=1, kind="oracle", host_cpu=model,
                nproc=usable, sample=f"{n}x{n} nodes of the same seeded planar tube, {more} steps, FP64, 1 thread")


def run_batch(precision: str, steps: int = 1000, n_tubes: int = 512, seed: int = 0, shape=None,
              graph: bool = True, keep_rho: bool = False):
    """512 seeded 1-D tubes in one pool: autotune (or the given tile shape),
    graph, time `steps` steps; with keep_rho also return every tube's
    density (slot order = tube order) after the run."""
    from paper_1602_02675_amd import inputs
    from paper_1602_02675_amd.lbsd import Pool

    lens = inputs.tube_lengths(seed, n_tubes)
    elem = 8 if precision == "fp64" else 4
    arena = int(sum(2 * (((3 * int(L) * elem) + 255) // 256 * 256) for L in lens)) + (1 << 20)
    pool = Pool(1, n_tubes, arena, precision=precision)
    for i, L in enumerate(lens):
        left, right, xd = inputs.riemann_instance(seed * 100000 + i)
        pool.admit_riemann(int(L), xd, left, right, steps + 10 ** 6, lam=inputs.cfl_lambda([left, right]))
    if shape is None:
        pool.advance(50)  # tuned on developed flows: the first steps after a Riemann start are not typical
        best, tuned_ms = pool.autotune(trials=5)
    else:
        pool.set_shape(shape)
        best = shape
    if graph:
        pool.use_graph(50)
    pool.advance(50)  # warm-up (and graph capture)
    ms = pool.advance_timed(steps)
    nodes = int(lens.sum())
    # densities of every tube after the run (untimed), for the FP32-vs-FP64 error
    rho = [pool.moments(slot)[0, 0] for slot in range(n_tubes)] if keep_rho else None
    pool.close()
    out = dict(value=round(nodes * steps / (ms * 1e-3) / 1e6, 1), unit="MLUPS", tubes=n_tubes, nodes=nodes,
               steps=steps, ms_per_step=round(ms / steps, 5), tile_shape=best,
               achieved_GBs=round(2 * 3 * elem * nodes / (ms * 1e-3 / steps) / 1e9, 1))
    return (out, rho) if keep_rho else out


def run_batch2d(precision: str, n: int = 48, steps: int = 250, seed: int = 5, keep_rho: bool = False):
    """Planar 2-D tubes of uneven sizes in one square-lattice pool."""
    from paper_1602_02675_amd import inputs
    from paper_1602_02675_amd.lbsd import Pool

    rng = np.random.default_rng(seed)
    nxs = np.rint(np.exp(rng.uniform(np.log(256), np.log(4096), size=n))).astype(int)
    nys = np.rint(np.exp(rng.uniform(np.log(64), np.log(1024), size=n))).astype(int)
    pool = Pool(2, n, 1 << 30, precision=precision)  # sized below
    need = sum(pool.footprint(int(a), int(b)) for a, b in zip(nxs, nys))
    pool.close()
    pool = Pool(2, n, need + (1 << 24), precision=precision)
    slots = []
    for i, (a, b) in enumerate(zip(nxs, nys)):
        left, right, xd = inputs.riemann_instance(seed * 100000 + i)
        sl = pool.admit_riemann(int(a), xd, left, right, steps + 10 ** 6, ny=int(b),
                                lam=inputs.cfl_lambda([left, right]))
        assert sl is not None, "the arena holds every tube"
        slots.append(sl)
    pool.advance(50)  # tuned on developed flows: the first steps after a Riemann start are not typical
    best, _ = pool.autotune(trials=5)
    pool.use_graph(25)
    pool.advance(50)  # warm-up (and graph capture)
    ms = pool.advance_timed(steps)
    nodes = int(np.sum(nxs * nys))
    rho = [pool.moments(sl)[0] for sl in slots] if keep_rho else None
    pool.close()
    elem = 8 if precision == "fp64" else 4
    out = dict(value=round(nodes * steps / (ms * 1e-3) / 1e6, 1), unit="MLUPS", tubes=n, nodes=nodes,
               steps=steps, ms_per_step=round(ms / steps, 5), tile_shape=best,
               achieved_GBs=round(2 * 4 * elem * nodes / (ms * 1e-3 / steps) / 1e9, 1))
    return (out, rho) if keep_rho else out


def run_serve(n_requests: int = 100, seed: int = 0):
    """Poisson arrivals at 0.5, 0.8 and 1.0 x measured capacity on an FP32
    square-lattice pool (the headline figures at 0.8)."""
    from paper_1602_02675_amd import inputs, serve
    from paper_1602_02675_amd.lbsd import Pool

    probe = inputs.serve_requests(seed, n_requests, rate_per_s=1.0)
    pool = Pool(2, 64, 24 << 30, precision="fp32")
    pool.use_graph(25)
    cap_nups, shape = serve.calibrate(pool, probe)
    mean_work = sum(r["side"] ** 2 * r["steps"] for r in probe) / len(probe)
    loads = {}
    for load in (0.5, 0.8, 1.0):
        rate = load * cap_nups / mean_work
        reqs = inputs.serve_requests(seed, n_requests, rate_per_s=rate)
        res = serve.run(pool, reqs, tick=25)
        offered = sum(r["side"] ** 2 * r["steps"] for r in reqs) / max(reqs[-1]["arrival"], 1e-9)
        loads[str(load)] = dict(rate_per_s=round(rate, 3), offered_MLUPS=round(offered / 1e6, 1),
                                served_MLUPS=round(res["nups"] / 1e6, 1), p50_latency_s=round(res["p50_s"], 4),
                                p99_latency_s=round(res["p99_s"], 4), makespan_s=round(res["makespan_s"], 3))
    # the same requests all queued at once: the served throughput at saturation
    sat = serve.run(pool, inputs.serve_requests(seed, n_requests, rate_per_s=1e9), tick=25)
    pool.close()
    at = loads["0.8"]
    return dict(value=at["served_MLUPS"], unit="MLUPS", requests=n_requests, load=0.8,
                rate_per_s=at["rate_per_s"], capacity_MLUPS=round(cap_nups / 1e6, 1),
                p50_latency_s=at["p50_latency_s"], p99_latency_s=at["p99_latency_s"], makespan_s=at["makespan_s"],
                loads=loads, tile_shape=shape, saturated_MLUPS=round(sat["nups"] / 1e6, 1),
                saturated_makespan_s=round(sat["makespan_s"], 3), precision="fp32")


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
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the walls, nonplanar, rest_level, tube1d(_fp32), two_gas and two_gas2d legs")
    ap.add_argument("--profile", action="store_true",
                    help="short run + a plain copy of known size, for rocprofv3 counters")
    ap.add_argument("--profile-batch", action="store_true",
                    help="as --profile, for the FP64 tube batch (tile shape 2, --steps steps)")
    ap.add_argument("--profile-hex", action="store_true",
                    help="as --profile, for the hexagonal-lattice tube (FP64, --steps steps)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(slabs along x with a halo exchange would be the multi-GPU design)", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.profile or args.profile_batch or args.profile_hex:
        # plain device copy of 1 GiB, three times (counter calibration)
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        if args.profile_batch:
            print(json.dumps({"profile": True, "batch": run_batch("fp64", steps=args.steps, shape=2, graph=False)}), flush=True)
            return
        if args.profile_hex:
            print(json.dumps({"profile": True, "hex": run_hex(args.steps)}), flush=True)
            return
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
                     "kernel": "march2d step: lean, short and full passes (march2d_lean_kernel<double>, "
                               "march2d_kernel<double, 3>, march2d_kernel<double, 5>)",
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
                       "rel_l1_density_vs_fp64_steps": args.warmup + args.steps,
                       "rel_l1_density_vs_fp64_2000_steps": fp32_accuracy(2000),
                       "rel_l1_density_vs_fp64_2000_steps_seeds_0_7": [fp32_accuracy(2000, seed=q)
                                                                        for q in range(8)],
                       "achieved_GBs": round(BYTES_PER_NODE["fp32"] * nodes /
                                             (r32["kernel_ms"] / 1e3 / args.steps) / 1e9, 1)}
    if not args.no_extra:
        rw = run_gpu("fp64", 500, args.warmup, bc_x="reflecting")
        out["walls"] = {"value": round(nodes * 500 / (rw["total_ms"] / 1e3) / 1e6, 1), "unit": "MLUPS",
                        "steps": 500, "ms_per_step": round(rw["total_ms"] / 500, 5),
                        "bc": "reflecting x / periodic y", "precision": "fp64"}
        out["nonplanar"] = run_nonplanar()
        out["hex"] = run_hex()
        rr = run_gpu("fp64", 100, 5, d0_frac=0.5)
        out["rest_level"] = {"value": round(nodes * 100 / (rr["total_ms"] / 1e3) / 1e6, 1), "unit": "MLUPS",
                             "steps": 100, "ms_per_step": round(rr["total_ms"] / 100, 5), "d0_frac": 0.5,
                             "precision": "fp64"}
        out["tube1d"] = run_tube1d()
        out["tube1d_fp32"] = run_tube1d(precision="fp32")
        out["two_gas"] = run_tube1d(gamma2=5.0 / 3.0)
        rg = run_gpu("fp64", 100, 5, gamma2=5.0 / 3.0)
        out["two_gas2d"] = {"value": round(nodes * 100 / (rg["total_ms"] / 1e3) / 1e6, 1), "unit": "MLUPS",
                            "steps": 100, "ms_per_step": round(rg["total_ms"] / 100, 5),
                            "gammas": [1.4, 5.0 / 3.0], "precision": "fp64"}
    if not args.no_batch:
        (b32, rho32), (b64, rho64) = (run_batch(p, keep_rho=True) for p in ("fp32", "fp64"))
        # the FP32 batch against the FP64 batch after the same steps: relative
        # L1 density error over all tubes (both batches ran the same steps: 50 developing,
        # 50 warm-up, 1000 timed)
        num = sum(float(np.sum(np.abs(a - b))) for a, b in zip(rho32, rho64))
        den = sum(float(np.sum(np.abs(b))) for b in rho64)
        b32["rel_l1_density_vs_fp64"] = num / den
        out["batch"] = {"fp32": b32, "fp64": b64}
        (c32, r32), (c64, r64) = (run_batch2d(p, keep_rho=True) for p in ("fp32", "fp64"))
        c32["rel_l1_density_vs_fp64"] = (sum(float(np.sum(np.abs(a - b))) for a, b in zip(r32, r64)) /
                                         sum(float(np.sum(np.abs(b))) for b in r64))
        out["batch2d"] = {"fp32": c32, "fp64": c64}
    if not args.no_serve:
        out["serve"] = run_serve()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_baseline_batch"] = cpu_baseline_batch()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: sub-step particle pushes per second of the sub-cycled Boris push.

Workload (one bench step = one pass of the whole hot path over one batch):
2^20 electrons at rest spread over 8 wavelengths in a linearly polarised
plane wave a = a0 sin(t - x), a0 = 150 (seed 22; seeds 20 and 21 give
a0 = 30 and 100), T/dt = 75, dx = 1.01 c dt (74.26 cells per wavelength),
8192 cells, 100 laser periods (7500 steps of dt), 3rd-order temporal
interpolation, psi_max = 0.01.  A step loads the initial state (device to
device), then runs all 7500 steps in launches of S steps, each launch
preceded by the on-device sampling of its field levels.

Printed: one JSON line with the metric, the roofline of the push kernel
(its average launch duration from HIP events on the push stream over the
timed region) and the FP64 CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6      # vector FP64, FMA counted as 2 flops
PEAK_HBM_GBS = 8000.0


def flops_per_substep(order: int) -> int:
    """Algorithmic FP64 operations of one sub-step (mul, add, div, sqrt = 1):
    grid coordinate 2, E tent 4p+8, B tent 4p+7, Boris 26, position 10."""
    return 8 * order + 53


FLOPS_PER_DECISION = 11       # grid coordinate 2, gamma 7, psi0 2
BYTES_PER_PARTICLE_STEP = 4 * 8 * 2 + 2 * 2   # x, px, py, pz read+write; k_old, status


def algorithmic_flops(counters: dict, order: int) -> int:
    f = flops_per_substep(order)
    return sum(c * (FLOPS_PER_DECISION + (4 ** k) * f) for k, c in enumerate(counters["steps_by_k"]))


def cpu_baseline(wl, every: int, threads: int):
    """FP64 oracle on every `every`-th particle over the full run."""
    from oracle import oracle as O
    from paper_2102_10983_amd import workloads as W
    if not os.path.exists(O.LIB_PATH):
        O.build()
    idx = np.arange(0, wl.num, every)
    table, M, shift = wl.table()
    fs = O.FieldSource(table=table, M=M, coeffs=W.shifted_coeffs(wl.lat, shift))
    prm = O.make_params(wl.ncells, wl.order, wl.dx, wl.dt, wl.psi_max, wl.x_origin)
    st = O.State(wl.x0[idx], wl.p0[0][idx], wl.p0[1][idx], wl.p0[2][idx])
    cnt = O.Counters()
    t0 = time.perf_counter()
    O.push(prm, fs, st, 0, wl.steps, counters=cnt, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": cnt.sub_steps / dt, "unit": "sub-step pushes/s", "cores": threads,
            "kind": "oracle",
            "sample": f"every {every}th electron ({len(idx)}) over the full {wl.steps} steps; "
                      f"{cnt.sub_steps} sub-steps in {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=22, choices=(20, 21, 22))
    ap.add_argument("--S", type=int, default=int(os.environ.get("PICSUB_BENCH_S", "0")),
                    help="steps of dt per push launch (0: the whole run in one launch)")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32c", "fp64fast"))
    ap.add_argument("--binning", default="none", choices=("none", "ballot", "learned"))
    ap.add_argument("--num", type=int, default=1 << 20)
    ap.add_argument("--periods", type=float, default=100.0)
    ap.add_argument("--cpu-every", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()

    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the push shards by particle index with no "
              "exchange, so only --gpus 1 is run here", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2102_10983_amd import runner, workloads as W

    wl = W.large_case(seed=args.seed, num=args.num, periods=args.periods)
    if args.S <= 0:
        args.S = wl.steps
    run = runner.DeviceRun(wl, S=args.S, precision=args.precision, binning=args.binning)
    stream = torch.cuda.current_stream()

    def one_step(events=None):
        run.reset()
        run.pusher.counters_reset()
        end = wl.steps
        while run.n < end:
            s = min(args.S, end - run.n)
            run.pusher.fields_load_lattice(run.n, s, run.table, run.M, run.coeffs)
            if events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                run.pusher.push(run.n, s)
                e1.record(stream)
                events.append((e0, e1))
            else:
                run.pusher.push(run.n, s)
            run.n += s

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    counters = run.pusher.counters()     # one full pass: counts per step

    events = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(events)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    if args.warmup == 0:
        counters = run.pusher.counters()
    sub_per_step = counters["sub_steps"]
    value = sub_per_step * args.steps / elapsed
    kernel_ms = sum(a.elapsed_time(b) for a, b in events)
    launches = len(events)
    avg_launch_s = kernel_ms / 1e3 / launches
    flops_step = algorithmic_flops(counters, wl.order)
    achieved = flops_step * args.steps / (kernel_ms / 1e3) / 1e12
    res = {
        "metric": "sub-step particle pushes/sec at rel err<=1e-5 vs FP64 oracle; "
                  "learned-binned vs plain",
        "value": value,
        "unit": "sub-step pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp64fast": "f64", "fp32c": "f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"plane wave a0={wl.a0:g}, {wl.num} electrons over 8 lambda, "
                               f"T/dt=75, dx=1.01 c dt, {wl.ncells} cells, {wl.steps} steps, "
                               f"order {wl.order}, psi_max {wl.psi_max}",
                   "precision": args.precision, "binning": args.binning,
                   "steps_per_launch": args.S, "sub_steps_per_pass": sub_per_step,
                   "mean_sub_steps_per_particle_step": sub_per_step / counters["steps"],
                   "n_star": counters["n_star"], "steps_by_k": counters["steps_by_k"][:9]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                     "kernel": {"fp64": "push_wave_kernel<3>", "fp64fast": "push_wave_fast_kernel<3>",
                                "fp32c": "push_wave_mixed_kernel<3>"}[args.precision]
                     if args.binning != "ballot" else "push_tile_kernel<3>", "launches": launches,
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "flops_per_launch": flops_step * args.steps / launches},
    }
    if not args.no_cpu:
        threads = len(os.sched_getaffinity(0))
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_every, threads)
    run.close()
    print(json.dumps(res))


if __name__ == "__main__":
    main()

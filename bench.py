"""Benchmark: sub-step particle pushes per second of the sub-cycled Boris push.

Workload (one bench step = one pass of the whole hot path over one batch):
2^20 electrons at rest spread over 8 wavelengths in a linearly polarised
plane wave a = a0 sin(t - x), a0 = 150 (seed 22; seeds 20 and 21 give
a0 = 30 and 100), T/dt = 75, dx = 1.01 c dt (74.26 cells per wavelength),
8192 cells, 100 laser periods (7500 steps of dt), 3rd-order temporal
interpolation, psi_max = 0.01.  A step loads the initial state (device to
device, sorted by position), with --binning learned scores every electron
with the load predictor and re-bins them (heaviest groups first), samples
the field levels on the device and runs all 7500 steps in launches of S
steps (default: one launch).

Printed: one JSON line with the metric, the same pass timed with plain
binning and with the plain FP64 (IEEE) push, the roofline of the push kernel
(its average launch duration from HIP events on the push stream over the
timed region) and the FP64 CPU oracle timed on a bounded sample.
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

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6      # vector FP64, FMA counted as 2 flops
PEAK_HBM_GBS = 8000.0

KERNELS = {  # (kernel name in traces, sources it is built from)
    "fp64": ("push_wave_kernel<3, 1, false, false>", ("push_wave.hpp", "common.hpp")),
    "fp64fast": ("push_fast_kernel<3, 1, false, false, 0>", ("push_fast.hpp", "common.hpp")),
    "fp64fast/occ5": ("push_fast_kernel<3, 1, false, false, 5>", ("push_fast.hpp", "common.hpp")),
    "fp32c": ("push_wave_fp32c_kernel<3, 1, false>", ("push_f32c.hpp", "push_fast.hpp",
                                                        "common.hpp")),
    "ballot": ("push_tile_kernel<3, 256, false>", ("push_tile.hpp", "common.hpp")),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "push_traffic.json")


def flops_per_substep(order: int) -> int:
    """Algorithmic FP64 operations of one sub-step (mul, add, div, sqrt = 1):
    grid coordinate 2, E tent 4p+8, B tent 4p+7, Boris 26, position 10."""
    return 8 * order + 53


FLOPS_PER_DECISION = 11       # grid coordinate 2, gamma 7, psi0 2


def algorithmic_flops(counters: dict, order: int) -> int:
    f = flops_per_substep(order)
    return sum(c * (FLOPS_PER_DECISION + (4 ** k) * f) for k, c in enumerate(counters["steps_by_k"]))


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2102_10983_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str, launches_per_step: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs, if they were taken on the kernel as built now."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh).get(key)
    name, files = KERNELS[key]
    if not rec or rec.get("source_hash") != source_hash(files):
        return None
    return rec["bytes_per_launch"] if launches_per_step == rec.get("launches_per_pass", 1) else None


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


class Pass:
    """One configuration of the hot path on one workload (a single run,
    host-driven launches of S steps) or on a batch of runs (device-driven
    windows of S steps, each run stopping at its own step count)."""

    def __init__(self, wl, S, precision, binning, predictor=None, fields="lattice",
                 occupancy=0):
        from paper_2102_10983_amd import runner
        self.wl = wl
        self.fill_events = []
        self.S = S
        self.binning = binning
        self.predictor = predictor
        self.pb_width = 0.0625
        kernel_binning = "ballot" if binning == "ballot" else "none"
        self.batch = isinstance(wl, list)
        if self.batch:
            self.run = runner.BatchRun(wl, S=S, precision=precision, binning=kernel_binning)
            self.pusher = self.run.pusher
            self.a0 = [w.a0 for w in wl]
        else:
            self.run = runner.DeviceRun(wl, S=S, precision=precision, binning=kernel_binning,
                                        fields=fields)
            self.pusher = self.run.pusher
            self.a0 = wl.a0
        if occupancy:
            self.pusher.tune_set(occupancy=occupancy)

    def step(self, stream=None, events=None):
        import torch
        run, wl = self.run, self.wl
        run.reset()
        self.pusher.counters_reset()
        if self.binning == "learned":
            self.predictor.prebin(self.pusher, self.a0, n=None if self.batch else 0,
                                  width=self.pb_width)
        if self.batch:
            for _ in range(run.windows):
                if events is not None:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    self.pusher.advance(self.S)
                    e1.record(stream)
                    events.append((e0, e1))
                else:
                    self.pusher.advance(self.S)
            return
        while run.n < wl.steps:
            s = min(self.S, wl.steps - run.n)
            if events is not None:
                f0 = torch.cuda.Event(enable_timing=True)
                f1 = torch.cuda.Event(enable_timing=True)
                f0.record(stream)
                run.fill(run.n, s)
                f1.record(stream)
                self.fill_events.append((f0, f1))
            else:
                run.fill(run.n, s)
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

    def time(self, steps, warmup, stream, events=None):
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step(stream, events)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def close(self):
        self.run.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=("large", "batch", "stress", "predictor"),
                    help="large: the default single run; batch: 64 uneven runs; stress: "
                         "thermal electrons over 200 wavelengths; predictor: 2^22 electrons at "
                         "rest on 16384 cells, the learned-binning workload")
    ap.add_argument("--seed", type=int, default=22, choices=(20, 21, 22))
    ap.add_argument("--psi", type=float, default=0.01, help="psi_max of the stress workload")
    ap.add_argument("--S", type=int, default=0,
                    help="steps of dt per push launch (0: the whole run in one launch)")
    ap.add_argument("--precision", default="fp64fast", choices=("fp64", "fp32c", "fp64fast"))
    ap.add_argument("--fields", default="lattice", choices=("lattice", "yee"),
                    help="large/stress: field levels sampled from the prescribed wave "
                         "(perfectly propagating PIC) or made by the Yee solver (standard PIC)")
    ap.add_argument("--binning", default="learned", choices=("none", "ballot", "learned"))
    ap.add_argument("--num", type=int, default=0,
                    help="electrons (large: 2^20, stress: 2^24, predictor: 2^22; batch: scale "
                         "factor x 1e6)")
    ap.add_argument("--periods", type=float, default=100.0)
    ap.add_argument("--order", type=int, default=3, choices=(1, 3, 5),
                    help="large/stress: temporal interpolation order p")
    ap.add_argument("--occupancy", default="auto", choices=("auto", "0", "5"),
                    help="register budget of the FP64_FAST push at orders 1, 3 (pic_tune): "
                         "auto times one untimed pass with each and keeps the faster")
    ap.add_argument("--pb-width", type=float, default=0.0625,
                    help="cost step (log2 sub-steps) of the learned group order")
    ap.add_argument("--cpu-every", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain-binning and plain-FP64 passes")
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
    from paper_2102_10983_amd import predictor as PR, workloads as W

    if args.workload == "large":
        wl = W.large_case(seed=args.seed, num=args.num or (1 << 20), periods=args.periods,
                          order=args.order)
        steps_max = wl.steps
        wdesc = (f"plane wave a0={wl.a0:g}, {wl.num} electrons at rest over 8 lambda, T/dt=75, "
                 f"dx=1.01 c dt, {wl.ncells} cells, {wl.steps} steps, order {wl.order}, "
                 f"psi_max {wl.psi_max}")
    elif args.workload == "predictor":
        wl = W.predictor_case(num=args.num or (1 << 22), periods=args.periods, order=args.order)
        steps_max = wl.steps
        wdesc = (f"plane wave a0=150, {wl.num} electrons at rest over 16 lambda, T/dt=75, "
                 f"{wl.ncells} cells, {wl.steps} steps, order {wl.order}, psi_max {wl.psi_max}")
    elif args.workload == "stress":
        wl = W.stress_case(psi_max=args.psi, num=args.num or (1 << 24), periods=args.periods,
                           order=args.order)
        steps_max = wl.steps
        wdesc = (f"plane wave a0=150, {wl.num} thermal (10 keV) electrons over 200 lambda, "
                 f"T/dt=75, {wl.ncells} cells, {wl.steps} steps, order {wl.order}, psi_max {wl.psi_max}")
    else:
        scale = (args.num / 1e6) if args.num else 1.0
        wl = W.batch_case(seed=3, nruns=64, periods=50.0, scale=scale)
        steps_max = max(w.steps for w in wl)
        wdesc = (f"64 runs, {sum(w.num for w in wl)} electrons (log-uniform 1e3..4e6 per run), "
                 f"a0 log-uniform 1..150, T/dt in {{40,75,150}}, 50 periods, order 3, psi_max 0.01")
    S = steps_max if args.S <= 0 else args.S
    model = PR.Predictor.load() if args.binning == "learned" else None
    stream = torch.cuda.current_stream()

    if args.workload == "batch" and args.fields != "lattice":
        print("the batch workload samples its fields on the device (--fields lattice)",
              file=sys.stderr)
        sys.exit(2)
    main_pass = Pass(wl, S, args.precision, args.binning, model, args.fields)
    main_pass.pb_width = args.pb_width
    order = wl[0].order if isinstance(wl, list) else wl.order
    occ_trials = None
    occupancy = 0
    if args.precision == "fp64fast" and order <= 3 and args.binning != "ballot":
        if args.occupancy == "auto":
            occ_trials = {}
            for occ in (0, 5):
                main_pass.pusher.tune_set(occupancy=occ)
                main_pass.step()                          # warm-up with this budget
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                main_pass.step()
                torch.cuda.synchronize()
                occ_trials[occ] = (time.perf_counter() - t0) * 1e3
            occupancy = min(occ_trials, key=occ_trials.get)
        else:
            occupancy = int(args.occupancy)
        main_pass.pusher.tune_set(occupancy=occupancy)
    events = []
    elapsed = main_pass.time(args.steps, args.warmup, stream, events)
    counters = main_pass.pusher.counters()              # the last pass
    main_pass.close()

    sub_per_step = counters["sub_steps"]
    value = sub_per_step * args.steps / elapsed
    kernel_ms = sum(a.elapsed_time(b) for a, b in events)
    launches = len(events)
    launches_per_step = launches // args.steps
    flops_step = algorithmic_flops(counters, order)
    achieved = flops_step * args.steps / (kernel_ms / 1e3) / 1e12
    key = "ballot" if args.binning == "ballot" else args.precision
    if key == "fp64fast" and occupancy == 5:
        key = "fp64fast/occ5"
    traffic = (measured_traffic(key, launches_per_step)
               if args.workload == "large" and args.fields == "lattice" and order == 3 else None)
    solve_ms = (sum(a.elapsed_time(b) for a, b in main_pass.fill_events) / args.steps
                if args.fields == "yee" else None)

    compare = []
    if not args.no_compare:
        legs = [("plain binning, same precision", args.precision, "none", args.fields),
                ("plain FP64 push (IEEE div/sqrt)", "fp64", "none", args.fields)]
        if args.workload == "large":
            other = "yee" if args.fields == "lattice" else "lattice"
            legs.append(({"yee": "standard PIC: levels from the Yee solver",
                          "lattice": "perfectly propagating PIC: levels sampled from the wave"}[other]
                         + ", same precision and binning", args.precision, args.binning, other))
        for label, prec, binning, fields in legs:
            if prec == args.precision and binning == args.binning and fields == args.fields:
                continue
            p = Pass(wl, S, prec, binning, model if binning == "learned" else None, fields,
                     occupancy if prec == "fp64fast" else 0)
            p.pb_width = args.pb_width
            ev = [] if fields == "yee" else None
            t = p.time(args.steps, args.warmup, stream, ev)
            c = p.pusher.counters()
            leg = {"label": label, "precision": prec, "binning": binning, "fields": fields,
                   "ms_per_step": t / args.steps * 1e3,
                   "value": c["sub_steps"] * args.steps / t,
                   "same_sub_steps": c["sub_steps"] == sub_per_step}
            if ev is not None:
                leg["push_ms"] = sum(a.elapsed_time(b) for a, b in ev) / args.steps
                leg["field_solve_ms"] = sum(a.elapsed_time(b) for a, b in p.fill_events) / args.steps
                leg["sub_steps_per_pass"] = c["sub_steps"]
            p.close()
            compare.append(leg)

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
        "config": {"workload": wdesc,
                   "precision": args.precision, "binning": args.binning, "fields": args.fields,
                   "steps_per_launch": S, "sub_steps_per_pass": sub_per_step,
                   "mean_sub_steps_per_particle_step": sub_per_step / counters["steps"],
                   "n_star": counters["n_star"], "steps_by_k": counters["steps_by_k"][:9],
                   "occupancy": occupancy,
                   **({"occupancy_trial_ms": occ_trials} if occ_trials else {}),
                   **({"field_solve_ms": solve_ms} if solve_ms is not None else {})},
        "compare": compare,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": KERNELS[key][0].replace("<3,", f"<{order},"), "launches": launches,
                     "avg_launch_ms": kernel_ms / launches,
                     "flops_per_launch": flops_step * args.steps / launches},
    }
    if not args.no_cpu and args.workload == "large" and args.fields == "lattice":
        threads = len(os.sched_getaffinity(0))
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_every, threads)
    print(json.dumps(res))


if __name__ == "__main__":
    main()

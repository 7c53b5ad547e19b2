"""Benchmark: sub-step particle pushes per second of the sub-cycled Boris push.

Workload (one bench step = one pass of the whole hot path over one batch),
by default the learned-binning configuration: 2^22 electrons at rest spread
over 16 wavelengths in a linearly polarised plane wave a = a0 sin(t - x),
a0 = 150, T/dt = 75, dx = 1.01 c dt (74.26 cells per wavelength), 16384
cells, 100 laser periods (7500 steps of dt), 3rd-order temporal
interpolation, psi_max = 0.01.  A step loads the initial state (device to
device, sorted by position), with --binning learned scores every electron
with the load predictor and orders the groups heaviest first, samples the
field levels on the device and runs all 7500 steps in launches of S steps
(default: one launch).

Printed: one JSON line with the metric (learned order), the same pass with
plain binning, with the plain FP64 (IEEE) push and with the FP32-compensated
push, the other workload shapes (2^20 electrons on 8192 cells; 64 uneven
runs; 2^24 thermal electrons) with the benchmark path, the roofline of the
push kernel (its average launch duration from HIP events on the push stream
over the timed region, against the algorithmic flop count), the FP64 CPU
oracle timed on a bounded sample (all host threads and one thread), and the
error of the benchmark path against the oracle on part of that sample.
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
    "fp64fast/occ6": ("push_fast_kernel<3, 1, false, false, 6>", ("push_fast.hpp", "common.hpp")),
    "fp64fast/occ7": ("push_fast_kernel<3, 1, false, false, 7>", ("push_fast.hpp", "common.hpp")),
    "fp32c": ("push_wave_fp32c_kernel<3, 1, false>", ("push_f32c.hpp", "push_fast.hpp",
                                                        "common.hpp")),
    "ballot": ("push_tile_kernel<3, 256, false>", ("push_tile.hpp", "common.hpp")),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "push_traffic.json")


# Algorithmic FP64 work (mul, add, div, sqrt counted 1, FMA 2): the tent
# gathers of E and B (11) and the Boris update with the position update (34)
# per sub-step, the decision's gather, gamma and psi0 (10) per step of dt.
FLOPS_PER_SUBSTEP = 45
FLOPS_PER_DECISION = 10


def algorithmic_flops(counters: dict) -> int:
    """Flops one pass needs by the algorithm's own count: 45 per sub-step
    (sum of 4^k over steps) + 10 per step."""
    return sum(c * (FLOPS_PER_DECISION + (4 ** k) * FLOPS_PER_SUBSTEP)
               for k, c in enumerate(counters["steps_by_k"]))


def model_flops_per_substep(order: int) -> int:
    """The flops the kernels' own formulation would need if every sub-step
    combined the p + 1 levels of E and B per particle: grid coordinate 2,
    E tent 4p+8, B tent 4p+7, Boris 26, position 10 (a k = 0 step reads E of
    level n directly, so this over-counts those)."""
    return 8 * order + 53


MODEL_FLOPS_PER_DECISION = 11       # grid coordinate 2, gamma 7, psi0 2


def model_flops(counters: dict, order: int) -> int:
    f = model_flops_per_substep(order)
    return sum(c * (MODEL_FLOPS_PER_DECISION + (4 ** k) * f)
               for k, c in enumerate(counters["steps_by_k"]))


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2102_10983_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_record(key: str, launches_per_step: int, workload: str, field: str):
    """A per-launch figure from the committed rocprofv3 runs (HBM bytes from
    FETCH_SIZE / WRITE_SIZE, VALU instructions from SQ_INSTS_VALU), if they
    were taken on this workload with the kernel as built now."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh).get(f"{key}@{workload}")
    name, files = KERNELS[key]
    if not rec or rec.get("source_hash") != source_hash(files):
        return None
    if launches_per_step != rec.get("launches_per_pass", 1):
        return None
    return rec.get(field)


def measured_traffic(key: str, launches_per_step: int, workload: str):
    """HBM bytes per launch (see measured_record)."""
    return measured_record(key, launches_per_step, workload, "bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, first: int, count: int, threads: int, one_thread: int, gpu=None,
                 check: int = 0):
    """The FP64 CPU oracle on `count` consecutive electrons (caller order:
    random positions) from `first`, over the full run, with all `threads`,
    then `one_thread` of them on one thread.  With gpu = (final device state,
    k trace of the first `check` electrons of the sample), also the error of
    the device run on those electrons (k-flip protocol: electrons whose k
    sequence differs are replayed by the oracle with the device's)."""
    from oracle import oracle as O
    from paper_2102_10983_amd import workloads as W
    if not os.path.exists(O.LIB_PATH):
        O.build()
    table, M, shift = wl.table()
    fs = O.FieldSource(table=table, M=M, coeffs=W.shifted_coeffs(wl.lat, shift))
    prm = O.make_params(wl.ncells, wl.order, wl.dx, wl.dt, wl.psi_max, wl.x_origin)

    def run(idx, nthreads, forced=None, trace=False):
        st = O.State(wl.x0[idx], wl.p0[0][idx], wl.p0[1][idx], wl.p0[2][idx])
        cnt = O.Counters()
        t0 = time.perf_counter()
        kt, pt = O.push(prm, fs, st, 0, wl.steps, counters=cnt, threads=nthreads,
                        forced_k=forced, trace=trace, psi_trace=trace)
        return st, cnt, time.perf_counter() - t0, kt, pt

    idx = np.arange(first, first + count)
    st, cnt, dt, _, _ = run(idx, threads)
    st1, cnt1, dt1, _, _ = run(idx[:one_thread], 1)
    out = {"value": cnt.sub_steps / dt, "unit": "sub-step pushes/s", "cores": threads,
           "kind": "oracle", "cpu": cpu_model(),
           "one_thread": {"value": cnt1.sub_steps / dt1, "cores": 1,
                          "sample": f"the first {one_thread} of those electrons, "
                                    f"{cnt1.sub_steps} sub-steps in {dt1:.2f} s"},
           "sample": f"{count} consecutive electrons (caller indices {first}..{first + count - 1}, "
                     f"random positions) over the full {wl.steps} steps; {cnt.sub_steps} "
                     f"sub-steps in {dt:.2f} s"}
    if gpu is None or check <= 0:
        return out, None
    d, gk = gpu
    cidx = idx[:check]
    ref, _, _, kt, pt = run(cidx, threads, trace=True)
    same = np.all(gk == kt, axis=0)
    flip_dist = 0.0
    for c in np.nonzero(~same)[0]:
        s0 = int(np.argmax(gk[:, c] != kt[:, c]))
        kk = max(int(gk[s0, c]), int(kt[s0, c]))
        flip_dist = max(flip_dist, abs(pt[s0, c] / 4.0 ** (kk - 1) - 1))
    if (~same).any():
        rep, _, _, _, _ = run(cidx[~same], threads, forced=np.ascontiguousarray(gk[:, ~same]))
        for key in ("x", "px", "py", "pz"):
            getattr(ref, key)[~same] = getattr(rep, key)
    gx, gpx, gpy, gpz = (d[k][cidx] for k in ("x", "px", "py", "pz"))
    dp = np.sqrt((gpx - ref.px) ** 2 + (gpy - ref.py) ** 2 + (gpz - ref.pz) ** 2)
    pref = np.sqrt(ref.px ** 2 + ref.py ** 2 + ref.pz ** 2)
    e_p = dp / np.maximum(pref, 1.0)
    e_x = np.abs(gx - ref.x) / np.maximum(np.abs(ref.x - wl.x0[cidx]), 2 * np.pi)
    g_gam = np.sqrt(1.0 + gpx ** 2 + gpy ** 2 + gpz ** 2)
    err = {"electrons": int(check), "max_e_p": float(e_p.max()),
           "p99_e_p": float(np.percentile(e_p, 99)), "max_e_x": float(e_x.max()),
           "max_e_gamma": float(np.max(np.abs(g_gam - ref.gamma()) / ref.gamma())),
           "max_e_px": float(np.max(np.abs(gpx - ref.px) / np.maximum(np.abs(ref.px), 1.0))),
           "k_flips": int((~same).sum()), "largest_flip_distance_from_threshold": flip_dist,
           "tolerance": 1e-5,
           "definition": "e_p = |p - p_ref| / max(|p_ref|, 1), e_x = |x - x_ref| / "
                         "max(|x_ref - x0|, 2 pi), e_gamma = |gamma - gamma_ref| / gamma_ref, "
                         "after the full run, caller indices from the cpu_baseline sample"}
    return out, err


class Pass:
    """One configuration of the hot path on one workload (a single run,
    host-driven launches of S steps) or on a batch of runs (device-driven
    windows of S steps, each run stopping at its own step count)."""

    def __init__(self, wl, S, precision, binning, predictor=None, fields="lattice",
                 occupancy=0, graph=False, reorder=False):
        from paper_2102_10983_amd import runner
        self.wl = wl
        self.graph = graph
        # single runs in windows: re-order the groups before every window by
        # the binning's score (learned, psi) or, for "persistence", by each
        # particle's load in the previous window (a k trace of it)
        self.reorder = reorder
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
        if graph:
            # a batch's whole pass (every window of every run) recorded once
            # as a HIP graph; each step replays it
            assert self.batch
            self.run.reset()
            self.run.capture()

    def step(self, stream=None, events=None):
        import torch
        run, wl = self.run, self.wl
        run.reset()
        self.pusher.counters_reset()
        if self.reorder and not self.batch:
            self._windows_reordered(stream, events)
            return
        if self.binning == "learned":
            self.predictor.prebin(self.pusher, self.a0, n=None if self.batch else 0,
                                  width=self.pb_width)
        elif self.binning == "psi":
            from paper_2102_10983_amd import predictor as PR
            score = PR.psi_score(self.pusher, self.a0, wl.dt, wl.psi_max, n=0)
            self.pusher.prebin(score, nbuckets=1, width=self.pb_width)
        if self.batch and self.graph:
            if events is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                run.replay()
                e1.record(stream)
                events.append((e0, e1))
            else:
                run.replay()
            return
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

    def _windows_reordered(self, stream, events):
        import torch
        from paper_2102_10983_amd import predictor as PR
        run, wl = self.run, self.wl
        buf = None
        if self.binning == "persistence":
            buf = torch.empty((self.S, wl.num), dtype=torch.int8, device="cuda")
        prev = None
        while run.n < wl.steps:
            s = min(self.S, wl.steps - run.n)
            if self.binning == "learned":
                self.predictor.prebin(self.pusher, self.a0, n=run.n, width=self.pb_width)
            elif self.binning == "psi":
                score = PR.psi_score(self.pusher, self.a0, wl.dt, wl.psi_max, n=run.n)
                self.pusher.prebin(score, nbuckets=1, width=self.pb_width)
            elif self.binning == "last_k":
                if run.n > 0:
                    self.pusher.prebin(PR.last_k_score(self.pusher), nbuckets=1,
                                       width=self.pb_width)
            elif self.binning == "persistence":
                if prev is not None:
                    self.pusher.prebin(PR.persistence_score(buf[:prev]), nbuckets=1,
                                       width=self.pb_width)
                self.pusher.ktrace_set(buf[:s], run.n, 0)
            run.fill(run.n, s)
            e0 = torch.cuda.Event(enable_timing=True) if events is not None else None
            e1 = torch.cuda.Event(enable_timing=True) if events is not None else None
            if e0:
                e0.record(stream)
            run.pusher.push(run.n, s)
            if e1:
                e1.record(stream)
                events.append((e0, e1))
            run.n += s
            prev = s
        if buf is not None:
            self.pusher.ktrace_set(None)

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
        if self.graph:
            self.pusher.graph_release()
        self.run.close()


OCC_BUDGETS = (0, 5, 6, 7)      # register budgets of the fast push (pic_tune.occupancy)


def trial_occupancy(p):
    """Time one untimed pass of p at each register budget (after one at that
    budget to warm up) and leave p at the fastest; (budget, {budget: ms})."""
    import torch
    trials = {}
    for occ in OCC_BUDGETS:
        p.pusher.tune_set(occupancy=occ)
        p.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.step()
        torch.cuda.synchronize()
        trials[occ] = (time.perf_counter() - t0) * 1e3
    best = min(trials, key=trials.get)
    p.pusher.tune_set(occupancy=best)
    return best, trials


def make_workload(name: str, args):
    """(workload, description) of one of the four workload shapes."""
    from paper_2102_10983_amd import workloads as W
    if name == "large":
        wl = W.large_case(seed=args.seed, num=args.num or (1 << 20), periods=args.periods,
                          order=args.order)
        desc = (f"plane wave a0={wl.a0:g}, {wl.num} electrons at rest over 8 lambda, T/dt=75, "
                f"dx=1.01 c dt, {wl.ncells} cells, {wl.steps} steps, order {wl.order}, "
                f"psi_max {wl.psi_max}")
    elif name == "predictor":
        wl = W.predictor_case(num=args.num or (1 << 22), periods=args.periods, order=args.order)
        desc = (f"learned-binning workload: plane wave a0=150, {wl.num} electrons at rest over "
                f"16 lambda, T/dt=75, dx=1.01 c dt, {wl.ncells} cells, {wl.steps} steps, "
                f"order {wl.order}, psi_max {wl.psi_max}")
    elif name == "stress20":
        wl = W.stress_case(psi_max=0.01, num=1 << 20, periods=100.0, order=3)
        desc = (f"plane wave a0=150, {wl.num} thermal (10 keV) electrons over 200 lambda, "
                f"T/dt=75, {wl.ncells} cells, {wl.steps} steps, order 3, psi_max 0.01")
    elif name == "stress":
        wl = W.stress_case(psi_max=args.psi, num=args.num or (1 << 24), periods=args.periods,
                           order=args.order)
        desc = (f"plane wave a0=150, {wl.num} thermal (10 keV) electrons over 200 lambda, "
                f"T/dt=75, {wl.ncells} cells, {wl.steps} steps, order {wl.order}, "
                f"psi_max {wl.psi_max}")
    else:
        scale = (args.num / 1e6) if args.num else 1.0
        wl = W.batch_case(seed=3, nruns=64, periods=50.0, scale=scale)
        desc = (f"64 runs, {sum(w.num for w in wl)} electrons (log-uniform 1e3..4e6 per run), "
                f"a0 log-uniform 1..150, T/dt in {{40,75,150}}, 50 periods, order 3, psi_max 0.01")
    return wl, desc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="predictor",
                    choices=("predictor", "large", "batch", "stress"),
                    help="predictor (default): 2^22 electrons at rest on 16384 cells, the "
                         "learned-binning workload; large: 2^20 electrons on 8192 cells; "
                         "batch: 64 uneven runs; stress: thermal electrons over 200 wavelengths")
    ap.add_argument("--seed", type=int, default=22, choices=(20, 21, 22),
                    help="large: a0 = 30, 100, 150 for seeds 20, 21, 22")
    ap.add_argument("--psi", type=float, default=0.01, help="psi_max of the stress workload")
    ap.add_argument("--S", type=int, default=0,
                    help="steps of dt per push launch (0: the whole run in one launch)")
    ap.add_argument("--precision", default="fp64fast", choices=("fp64", "fp32c", "fp64fast"))
    ap.add_argument("--fields", default="lattice", choices=("lattice", "yee"),
                    help="single runs: field levels sampled from the prescribed wave "
                         "(perfectly propagating PIC) or made by the Yee solver (standard PIC)")
    ap.add_argument("--binning", default="learned", choices=("none", "ballot", "learned", "psi"),
                    help="group order: slot (position) order, the compaction kernel, the "
                         "learned load predictor, or the step-0 value of the Psi criterion "
                         "(a non-learned control)")
    ap.add_argument("--num", type=int, default=0,
                    help="electrons (large: 2^20, stress: 2^24, predictor: 2^22; batch: scale "
                         "factor x 1e6)")
    ap.add_argument("--periods", type=float, default=100.0)
    ap.add_argument("--order", type=int, default=3, choices=(1, 2, 3, 5),
                    help="single runs: temporal interpolation order p")
    ap.add_argument("--occupancy", default="auto", choices=("auto", "0", "5", "6", "7"),
                    help="register budget of the FP64_FAST push at orders 1, 3 (pic_tune): "
                         "auto times one untimed pass with each and keeps the faster")
    ap.add_argument("--pb-width", type=float, default=0.0625,
                    help="cost step (log2 sub-steps) of the learned group order")
    ap.add_argument("--cpu-count", type=int, default=65536,
                    help="electrons in the oracle's timed sample (all host threads)")
    ap.add_argument("--cpu-one-thread", type=int, default=2048,
                    help="electrons of that sample timed again on one thread")
    ap.add_argument("--check", type=int, default=4096,
                    help="electrons of that sample whose error against the oracle is reported")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip every compare leg (other binning, precisions, workloads)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the compare legs on the other workload shapes")
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
    from paper_2102_10983_amd import predictor as PR

    wl, wdesc = make_workload(args.workload, args)
    batch = isinstance(wl, list)
    steps_max = max(w.steps for w in wl) if batch else wl.steps
    S = steps_max if args.S <= 0 else args.S
    model = PR.Predictor.load() if args.binning == "learned" or not args.no_compare else None
    stream = torch.cuda.current_stream()

    if batch and args.fields != "lattice":
        print("the batch workload samples its fields on the device (--fields lattice)",
              file=sys.stderr)
        sys.exit(2)
    main_pass = Pass(wl, S, args.precision, args.binning, model, args.fields)
    main_pass.pb_width = args.pb_width
    order = wl[0].order if batch else wl.order
    occ_trials = None
    occupancy = 0
    if args.precision == "fp64fast" and order <= 3 and args.binning != "ballot":
        if args.occupancy == "auto":
            occupancy, occ_trials = trial_occupancy(main_pass)
        else:
            occupancy = int(args.occupancy)
        main_pass.pusher.tune_set(occupancy=occupancy)
    events = []
    elapsed = main_pass.time(args.steps, args.warmup, stream, events)
    counters = main_pass.pusher.counters()              # the last pass
    sub_per_step = counters["sub_steps"]
    value = sub_per_step * args.steps / elapsed
    kernel_ms = sum(a.elapsed_time(b) for a, b in events)
    launches = len(events)
    launches_per_step = launches // args.steps
    flops_step = algorithmic_flops(counters)
    model_step = model_flops(counters, order)
    achieved = flops_step * args.steps / (kernel_ms / 1e3) / 1e12
    key = "ballot" if args.binning == "ballot" else args.precision
    if key == "fp64fast" and occupancy:
        key = f"fp64fast/occ{occupancy}"
    traffic = (measured_traffic(key, launches_per_step, args.workload)
               if args.fields == "lattice" and order == 3 and not args.num and args.periods == 100.0
               else None)
    solve_ms = (sum(a.elapsed_time(b) for a, b in main_pass.fill_events) / args.steps
                if args.fields == "yee" else None)

    # untimed: one more pass with the k trace of the electrons whose error
    # against the oracle is reported (the trace changes no result)
    do_cpu = not args.no_cpu and not batch and args.fields == "lattice"
    first = 0
    gpu_check = None
    if do_cpu:
        count = min(args.cpu_count, wl.num)
        first = int(np.random.default_rng(2024).integers(0, wl.num - count + 1))
        check = min(args.check, count)
        buf = torch.full((wl.steps, check), -2, dtype=torch.int8, device="cuda")
        main_pass.pusher.ktrace_set(buf, 0, first)
        main_pass.step()
        torch.cuda.synchronize()
        main_pass.pusher.ktrace_set(None)
        traced_counters = main_pass.pusher.counters()
        gpu_check = (main_pass.pusher.diag(), buf.cpu().numpy())
        assert traced_counters == counters, "a traced pass must take the same steps"
        del buf
    main_pass.close()

    compare = []
    if not args.no_compare:
        # label, workload, precision, binning, fields, timed steps[, steps per
        # launch, graph]
        legs = [("plain binning, same precision", args.workload, args.precision, "none",
                 args.fields, args.steps),
                ("groups ordered by the step-0 Psi criterion (non-learned control), same "
                 "precision", args.workload, args.precision, "psi", args.fields, args.steps),
                ("plain FP64 push (IEEE div/sqrt)", args.workload, "fp64", "none", args.fields,
                 args.steps),
                ("FP32-compensated push, same binning", args.workload, "fp32c", args.binning,
                 args.fields, args.steps),
                ("compaction by k alone: the ballot kernel (per-step ballot + per-k LDS "
                 "queues, IEEE FP64)", args.workload, "fp64", "ballot", args.fields, 1)]
        if args.workload == "large":
            other = "yee" if args.fields == "lattice" else "lattice"
            legs.append(({"yee": "standard PIC: levels from the Yee solver",
                          "lattice": "perfectly propagating PIC: levels sampled from the wave"}[other]
                         + ", same precision and binning", "large", args.precision, args.binning,
                         other, args.steps))
        if not args.no_configs and not args.num and args.periods == 100.0:
            for name in ("large", "batch", "stress"):
                if name != args.workload:
                    legs.append((f"workload {name}, same precision and binning", name,
                                 args.precision, args.binning, "lattice", 1))
                    if name == "stress":
                        legs.append((f"workload {name}, plain binning", name, args.precision,
                                     "none", "lattice", 1))
                        legs.append((f"workload {name}, step-0 Psi order", name,
                                     args.precision, "psi", "lattice", 1))
                    if name == "stress":
                        for b, what in (("none", "position order"),
                                        ("learned", "learned score before every window"),
                                        ("psi", "step-0 Psi score before every window"),
                                        ("last_k", "persistence: each particle's k at the "
                                                   "end of the previous window"),
                                        ("persistence", "persistence: each particle's load "
                                                        "in the previous window (k trace)")):
                            legs.append((f"2^20 thermal electrons in windows of 750 steps, {what}",
                                         "stress20", args.precision, b, "lattice", 1, 750,
                                         False, True))
                    if name == "batch":
                        legs.append(("workload batch in device-driven windows of 750 steps, "
                                     "the whole pass replayed from one HIP graph (rings of 753 "
                                     "levels instead of every level of a run)", name,
                                     args.precision, args.binning, "lattice", 1, 750, True))
        for leg_spec in legs:
            label, wname, prec, binning, fields, nsteps = leg_spec[:6]
            leg_S, leg_graph = (leg_spec[6], leg_spec[7]) if len(leg_spec) > 6 else (0, False)
            leg_reorder = leg_spec[8] if len(leg_spec) > 8 else False
            if (wname == args.workload and prec == args.precision and binning == args.binning
                    and fields == args.fields):
                continue
            if binning == "psi" and wname == "batch":
                continue
            lwl, ldesc = (wl, wdesc) if wname == args.workload else make_workload(wname, args)
            lsteps = max(w.steps for w in lwl) if isinstance(lwl, list) else lwl.steps
            p = Pass(lwl, leg_S or (lsteps if args.S <= 0 else args.S), prec, binning,
                     model if binning == "learned" else None, fields,
                     occupancy if prec == "fp64fast" else 0, graph=leg_graph,
                     reorder=leg_reorder)
            p.pb_width = args.pb_width
            leg_occ = occupancy if prec == "fp64fast" else 0
            lorder = lwl[0].order if isinstance(lwl, list) else lwl.order
            if (prec == "fp64fast" and lorder <= 3 and binning != "ballot" and not leg_graph
                    and args.occupancy == "auto"):
                leg_occ, _ = trial_occupancy(p)      # each leg at its own fastest budget
            ev = []
            t = p.time(nsteps, 1, stream, ev)
            c = p.pusher.counters()
            leg = {"label": label, "workload": ldesc if wname != args.workload else args.workload,
                   "precision": prec, "binning": binning, "fields": fields,
                   **({"steps_per_launch": leg_S, "hip_graph": True} if leg_graph else {}),
                   **({"steps_per_launch": leg_S, "reordered_every_window": True}
                      if leg_reorder else {}),
                   "steps": nsteps, "ms_per_step": t / nsteps * 1e3,
                   "value": c["sub_steps"] * nsteps / t,
                   "push_ms": sum(a.elapsed_time(b) for a, b in ev) / nsteps,
                   "sub_steps_per_pass": c["sub_steps"],
                   **({"occupancy": leg_occ} if prec == "fp64fast" else {})}
            if wname == args.workload:
                leg["same_sub_steps"] = c["sub_steps"] == sub_per_step
            if fields == "yee":
                leg["field_solve_ms"] = sum(a.elapsed_time(b) for a, b in p.fill_events) / nsteps
            p.close()
            compare.append(leg)

    # the attainable FP64 vector rate on this device (FMA chains, 16 per lane,
    # 32 waves per CU), best of three launches after one to warm up
    from paper_2102_10983_amd import picsub as PS
    PS.fma_probe(2048, 1000)
    attainable = max(PS.fma_probe(2048, 100000) for _ in range(3))
    # VALU issue bound: the push launch's wave-level VALU instructions (from
    # the committed rocprofv3 SQ_INSTS_VALU count of this kernel on this
    # workload), 4 cycles each on one of 1024 SIMDs at 2.4 GHz
    valu = (measured_record(key, launches_per_step, args.workload, "valu_instr_per_launch")
            if traffic is not None else None)
    ieee = [c for c in compare if c["precision"] == "fp64" and c["binning"] == "none"
            and c["workload"] == args.workload]
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
                   "n_star": counters["n_star"], "steps_by_k": counters["steps_by_k"][:13],
                   "clamps": counters["clamps"], "lost": counters["lost"],
                   "occupancy": occupancy,
                   **({"occupancy_trial_ms": occ_trials} if occ_trials else {}),
                   **({"field_solve_ms": solve_ms} if solve_ms is not None else {})},
        "compare": compare,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": KERNELS[key][0].replace("<3,", f"<{order},"), "launches": launches,
                     "avg_launch_ms": kernel_ms / launches,
                     "flops_per_launch": flops_step * args.steps / launches,
                     "flop_count": f"algorithmic: {FLOPS_PER_SUBSTEP} per sub-step, "
                                   f"{FLOPS_PER_DECISION} per step of dt",
                     "model_flops_per_launch": model_step * args.steps / launches,
                     "model_frac": model_step * args.steps / (kernel_ms / 1e3) / 1e12
                                   / PEAK_FP64_TFLOPS,
                     "attainable_peak": attainable,
                     "frac_attainable": achieved / attainable,
                     "attainable_from": "FMA-chain probe: 2048 x 256 lanes, 16 chains of 1e5 "
                                        "FMAs each, best of 3",
                     "valu_issue_frac": (valu * 4 / (1024 * 2.4e9)) / (kernel_ms / launches / 1e3)
                                        if valu else None},
        "speedup_vs_plain_fp64": (value / ieee[0]["value"]) if ieee else None,
    }
    if do_cpu:
        threads = len(os.sched_getaffinity(0))
        cpu, err = cpu_baseline(wl, first, min(args.cpu_count, wl.num), threads,
                                min(args.cpu_one_thread, args.cpu_count), gpu_check,
                                min(args.check, args.cpu_count))
        res["cpu_baseline"] = cpu
        res["error_vs_oracle"] = err
    print(json.dumps(res))


if __name__ == "__main__":
    main()

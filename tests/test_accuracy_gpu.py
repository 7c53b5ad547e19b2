"""Accuracy of the benchmark path (FP64 with refined hardware reciprocal and
rsqrt, learned group order, whole runs per launch) against the FP64 oracle
on the other workload shapes: thermal electrons over 200 wavelengths and a
batch of uneven runs.  Tolerance: 1e-5 relative on p and x with the k-flip
protocol of tests/parity.py; the measured errors are printed."""

import sys

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("num,psi", [(1 << 20, 0.01), (1 << 24, 0.01), (1 << 24, 0.003)],
                         ids=["2p20-psi0.01", "2p24-psi0.01", "2p24-psi0.003"])
def test_thermal_load_subsample(torch_gpu, num, psi):
    """Thermal electrons (10 keV) over 200 wavelengths, a0 = 150, 100 periods,
    learned order: 2^20 at Psi_max = 0.01 and the full 2^24 at 0.01 and
    0.003; 4096 consecutive electrons (caller order) checked against the
    oracle."""
    torch = torch_gpu
    from paper_2102_10983_amd import predictor, runner
    from parity import compare
    wl = W.stress_case(num=num, psi_max=psi)
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")
    run.reset()
    predictor.Predictor.load().prebin(run.pusher, wl.a0, n=0)
    first = int(np.random.default_rng(5).integers(0, wl.num - 4096))
    buf = torch.full((wl.steps, 4096), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, first)
    run.advance(wl.steps)
    d = run.diag()
    run.close()
    idx = np.arange(first, first + 4096)
    full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
    full[:, idx] = buf.cpu().numpy()
    res = compare(wl, wl.steps, d, idx, TOL, g_ktrace=full, flip_rel=1e-9)
    _say(f"thermal {num} psi {psi}:", {k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["max_e_p"] < 1e-6     # the bar is 1e-5


@pytest.mark.parametrize("run_index", [0, 17, 41])
def test_batch_runs(torch_gpu, run_index):
    """A scaled-down batch (64 runs, ~4e5 electrons, 50 periods, one window
    per run), learned order; up to 512 electrons of one run checked."""
    torch = torch_gpu
    from paper_2102_10983_amd import predictor, runner
    from parity import compare
    wls = W.batch_case(seed=3, nruns=64, periods=50.0, scale=0.02)
    S = max(w.steps for w in wls)
    br = runner.BatchRun(wls, S=S, precision="fp64fast", binning="none")
    br.reset()
    predictor.Predictor.load().prebin(br.pusher, [w.a0 for w in wls])
    wl = wls[run_index]
    off = int(sum(w.num for w in wls[:run_index]))
    m = min(512, wl.num)
    buf = torch.full((wl.steps, m), -2, dtype=torch.int8, device="cuda")
    br.pusher.ktrace_set(buf, 0, off)
    br.run_all()
    d = br.diag()
    br.close()
    sub = {k: d[k][off:off + wl.num] for k in ("x", "px", "py", "pz", "status")}
    full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
    full[:, :m] = buf.cpu().numpy()
    res = compare(wl, wl.steps, sub, np.arange(m), TOL, g_ktrace=full, flip_rel=1e-9)
    _say(f"batch run {run_index} ({wl.name}, {wl.num} electrons):",
         {k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["max_e_p"] < 1e-6     # the bar is 1e-5


def test_batch_full_scale_sampled(torch_gpu):
    """The full batch (64 uneven runs, 2.0e7 electrons, 50 periods each, one
    window per run, learned order): up to 4096 electrons of each of three
    runs of different a0 and T/dt against the oracle."""
    torch = torch_gpu
    from paper_2102_10983_amd import predictor, runner
    from parity import compare
    wls = W.batch_case(seed=3, nruns=64, periods=50.0)
    S = max(w.steps for w in wls)
    br = runner.BatchRun(wls, S=S, precision="fp64fast", binning="none")
    br.reset()
    predictor.Predictor.load().prebin(br.pusher, [w.a0 for w in wls])
    picks = (5, 29, 52)
    bufs = []
    for r in picks:
        wl = wls[r]
        off = int(sum(w.num for w in wls[:r]))
        m = min(4096, wl.num)
        buf = torch.full((wl.steps, m), -2, dtype=torch.int8, device="cuda")
        bufs.append((r, off, m, buf))
    # one trace buffer at a time: run the pass once per sampled run
    out = []
    for r, off, m, buf in bufs:
        br.reset()
        predictor.Predictor.load().prebin(br.pusher, [w.a0 for w in wls])
        br.pusher.ktrace_set(buf, 0, off)
        br.run_all()
        out.append((r, off, m, buf.cpu().numpy(), br.diag()))
    br.close()
    for r, off, m, kt, d in out:
        wl = wls[r]
        sub = {k: d[k][off:off + wl.num] for k in ("x", "px", "py", "pz", "status")}
        full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
        full[:, :m] = kt
        res = compare(wl, wl.steps, sub, np.arange(m), TOL, g_ktrace=full, flip_rel=1e-9)
        _say(f"full batch run {r} ({wl.name}, {wl.num} electrons):",
             {k: v for k, v in res.items() if k != "oracle_counters"})


def test_benchmark_configuration_sampled(torch_gpu):
    """The large case as its bench leg runs it: 2^20 electrons, a0 = 150,
    learned group order, the six-wavefront register budget its trial picks,
    7500 steps in one launch; 2048 consecutive electrons against the
    oracle."""
    torch = torch_gpu
    from paper_2102_10983_amd import predictor, runner
    from parity import compare
    wl = W.large_case(seed=22)
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")
    run.pusher.tune_set(occupancy=6)
    run.reset()
    predictor.Predictor.load().prebin(run.pusher, wl.a0, n=0)
    first = int(np.random.default_rng(23).integers(0, wl.num - 2048))
    buf = torch.full((wl.steps, 2048), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, first)
    run.advance(wl.steps)
    d = run.diag()
    run.close()
    idx = np.arange(first, first + 2048)
    full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
    full[:, idx] = buf.cpu().numpy()
    res = compare(wl, wl.steps, d, idx, TOL, g_ktrace=full, flip_rel=1e-9)
    _say("benchmark configuration:", {k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["max_e_p"] < 1e-6     # the bar is 1e-5


def test_predictor_workload_sampled(torch_gpu):
    """Exactly what bench.py times by default, the learned-binning workload:
    2^22 electrons at rest over 16 wavelengths, a0 = 150, 16384 cells, 100
    periods in one launch, learned order, the seven-wavefront register
    budget its trial picks; 2048 consecutive electrons against the oracle."""
    torch = torch_gpu
    from paper_2102_10983_amd import predictor, runner
    from parity import compare
    wl = W.predictor_case()
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")
    run.pusher.tune_set(occupancy=7)
    run.reset()
    predictor.Predictor.load().prebin(run.pusher, wl.a0, n=0)
    first = int(np.random.default_rng(29).integers(0, wl.num - 2048))
    buf = torch.full((wl.steps, 2048), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, first)
    run.advance(wl.steps)
    d = run.diag()
    run.close()
    idx = np.arange(first, first + 2048)
    full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
    full[:, idx] = buf.cpu().numpy()
    res = compare(wl, wl.steps, d, idx, TOL, g_ktrace=full, flip_rel=1e-9)
    _say("predictor workload:", {k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["max_e_p"] < 1e-6     # the bar is 1e-5

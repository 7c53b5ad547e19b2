"""The predictor attached to a context (pic_predictor_set): the pushes
score the particles and re-order the groups by themselves.

* Single run, host-driven launches, 2^20 thermal electrons at a0 = 150:
  the same bits as the plain push, one re-ordering per pass, and the same
  gain over position order as the caller-driven pic_prebin.
* Batch, device-driven windows (pic_advance): a re-ordering every second
  window, the same bits as the batch without a predictor.
* Argument errors; detaching stops the re-ordering.
"""

import sys
import time

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(d):
    return {k: d[k].copy() for k in ("x", "px", "py", "pz", "k_last", "status")}


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


def test_attached_predictor_on_a_thermal_load(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import predictor, runner
    model = predictor.Predictor.load()
    wl = W.stress_case(num=1 << 20)
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")

    def one(mode):
        run.reset()
        if mode == "manual":
            model.prebin(run.pusher, wl.a0, n=0)
        elif mode == "attached":
            model.attach(run.pusher, wl.a0, every=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.advance(wl.steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        if mode == "attached":
            run.pusher.predictor_set()                 # detach
        return t, run.diag()

    one("plain")                                       # warm-up
    res = {m: [one(m) for _ in range(2)] for m in ("plain", "manual", "attached")}
    best = {m: min(t for t, _ in v) for m, v in res.items()}
    _say({m: round(v * 1e3, 1) for m, v in best.items()})
    ref = res["plain"][-1][1]
    for m in ("manual", "attached"):
        got = res[m][-1][1]
        assert _same(_state(got), _state(ref)), m
    assert res["attached"][-1][1]["counters"]["rebins"] == 1
    assert res["manual"][-1][1]["counters"]["rebins"] == 0
    assert best["attached"] < 0.9 * best["plain"]
    run.close()


def test_attached_predictor_in_device_driven_windows(torch_gpu):
    from paper_2102_10983_amd import predictor, runner
    model = predictor.Predictor.load()
    wls = W.batch_case(seed=7, nruns=5, periods=3.0, p_range=(50, 3000),
                       a0_range=(5.0, 150.0), cells_range=(400, 900))
    ref = runner.BatchRun(wls, S=37, precision="fp64fast")
    ref.reset()
    ref.run_all()
    want = _state(ref.diag())
    ref.close()
    b = runner.BatchRun(wls, S=37, precision="fp64fast")
    b.reset()
    model.attach(b.pusher, [w.a0 for w in wls], every=2)
    b.run_all()
    got = b.diag()
    b.close()
    assert _same(_state(got), want)
    assert got["counters"]["rebins"] == (b.windows + 1) // 2


def test_predictor_set_arguments(torch_gpu):
    from paper_2102_10983_amd import picsub, predictor, runner
    model = predictor.Predictor.load()
    wl = W.small_case(order=3, num=512, periods=2)
    run = runner.DeviceRun(wl, S=10, precision="fp64fast", binning="none")
    run.reset()
    with pytest.raises(picsub.PicError):
        model.attach(run.pusher, wl.a0, every=0)
    with pytest.raises(picsub.PicError):
        model.attach(run.pusher, -1.0)
    model.attach(run.pusher, wl.a0, every=3)
    run.advance(50)                                    # five calls: turns at 1 and 4
    assert run.diag()["counters"]["rebins"] == 2
    run.pusher.predictor_set()
    run.advance(50)
    assert run.diag()["counters"]["rebins"] == 2
    run.close()


def test_attached_predictor_with_a_held_graph(torch_gpu):
    """While a captured graph is held, eager windows run without the
    predictor's turns (re-binning is not allowed then) instead of failing."""
    from paper_2102_10983_amd import predictor, runner
    model = predictor.Predictor.load()
    wls = W.batch_case(seed=8, nruns=3, periods=2.0, p_range=(50, 800),
                       a0_range=(5.0, 100.0), cells_range=(400, 700))
    b = runner.BatchRun(wls, S=30, precision="fp64fast")
    b.reset()
    model.attach(b.pusher, [w.a0 for w in wls], every=1)
    b.capture()
    b.run_all()                                        # eager windows, graph held
    assert b.diag()["counters"]["rebins"] == 0
    b.pusher.graph_release()
    b.reset()
    b.run_all()
    assert b.diag()["counters"]["rebins"] == b.windows
    b.close()

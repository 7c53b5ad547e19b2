"""What the trained load predictor gains over the method without it, and
over a non-learned score.

Thermal (10 keV) electrons in an a0 = 150 plane wave, spread over 200
wavelengths: the sub-cycling load differs from particle to particle and is
not ordered by position, so some 64-lane groups carry far more sub-steps
than others.  The plain push starts groups in position order; with the
learned order the heaviest groups (by the network's prediction from the
initial state) start first.  Psi still decides every step, so the results
are the same bit for bit; only the wall time changes.
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


def test_learned_order_beats_position_order_on_a_thermal_load():
    """Group orders on the 2^20 thermal load: position (plain), the step-0
    value of the Psi criterion (a non-learned control that knows each
    particle's next-step load exactly), the learned prediction of the whole
    run's load, and the true whole-run load of every particle taken from a
    traced pass (the best any score can do).  Same bits under every order;
    the learned order beats plain by 10 % and the non-learned control."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_10983_amd import predictor, runner
    model = predictor.Predictor.load()
    wl = W.stress_case(num=1 << 20)
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")

    def one(order):
        run.reset()
        if order == "learned":
            model.prebin(run.pusher, wl.a0, n=0)
        elif order == "psi":
            run.pusher.prebin(predictor.psi_score(run.pusher, wl.a0, wl.dt, wl.psi_max, n=0),
                              nbuckets=1, width=0.0625)
        elif order == "true":
            run.pusher.prebin(true, nbuckets=1, width=0.0625)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.advance(wl.steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    run.reset()
    tot = predictor.traced_load(run, wl.steps)
    true = torch.log2(tot.double().clamp(min=1) / wl.steps).float().contiguous()
    true[tot == 0] = float("nan")
    one("plain")                                 # warm-up
    plain = min(one("plain") for _ in range(3))
    ref = run.diag()
    times = {"plain": plain}
    for order in ("psi", "learned", "true"):
        times[order] = min(one(order) for _ in range(3))
        got = run.diag()
        for k in ("x", "px", "py", "pz", "k_last", "status"):
            assert np.array_equal(got[k], ref[k]), (order, k)
        assert got["counters"] == ref["counters"], order
    run.close()
    _say({k: f"{v * 1e3:.1f} ms" for k, v in times.items()})
    assert times["learned"] < 0.9 * times["plain"]
    assert times["learned"] < times["psi"]

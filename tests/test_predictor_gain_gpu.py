"""What the trained load predictor gains over the method without it.

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
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_10983_amd import predictor, runner
    model = predictor.Predictor.load()
    wl = W.stress_case(num=1 << 20)
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")

    def one(learned):
        run.reset()
        if learned:
            model.prebin(run.pusher, wl.a0, n=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.advance(wl.steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    one(False)                                  # warm-up
    plain = [one(False) for _ in range(3)]
    ref = run.diag()
    learned = [one(True) for _ in range(3)]
    got = run.diag()
    run.close()
    _say(f"plain {min(plain) * 1e3:.1f} ms, learned {min(learned) * 1e3:.1f} ms")
    for k in ("x", "px", "py", "pz", "k_last", "status"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["counters"] == ref["counters"]
    assert min(learned) < 0.9 * min(plain)

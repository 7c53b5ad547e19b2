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


def test_orders_in_windows_including_persistence():
    """The same load in launches of 750 steps, the groups re-ordered before
    every window: by position (none), by the learned score, by the step-0
    Psi score, and by two persistence controls: each particle's k at the
    last step of the previous window (free: it is in the state), and its
    mean load over the previous window from a k trace (which the push pays
    for with one byte store per particle and step).  Same bits under every
    order; the learned and Psi scores beat position order (the persistence
    timings are printed, not asserted)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_10983_amd import predictor, runner
    model = predictor.Predictor.load()
    wl = W.stress_case(num=1 << 20)
    S = 750
    run = runner.DeviceRun(wl, S=S, precision="fp64fast", binning="none")
    buf = torch.empty((S, wl.num), dtype=torch.int8, device="cuda")

    def one(order):
        run.reset()
        run.pusher.counters_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prev = None
        while run.n < wl.steps:
            s = min(S, wl.steps - run.n)
            if order == "learned":
                model.prebin(run.pusher, wl.a0, n=run.n)
            elif order == "psi":
                run.pusher.prebin(predictor.psi_score(run.pusher, wl.a0, wl.dt, wl.psi_max,
                                                      n=run.n), nbuckets=1, width=0.0625)
            elif order == "last k" and run.n > 0:
                run.pusher.prebin(predictor.last_k_score(run.pusher), nbuckets=1, width=0.0625)
            elif order == "trace":
                if prev is not None:
                    run.pusher.prebin(predictor.persistence_score(buf[:prev]), nbuckets=1,
                                      width=0.0625)
                run.pusher.ktrace_set(buf[:s], run.n, 0)
            run.advance(s)
            prev = s
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        run.pusher.ktrace_set(None)
        d = run.diag()
        return t, d

    res = {o: one(o) for o in ("none", "learned", "psi", "last k", "trace")}
    run.close()
    _say({o: f"{t * 1e3:.1f} ms" for o, (t, _) in res.items()})
    ref = res["none"][1]
    for o, (t, d) in res.items():
        for key in ("x", "px", "py", "pz", "k_last", "status"):
            assert np.array_equal(d[key], ref[key]), (o, key)
        assert d["counters"]["sub_steps"] == ref["counters"]["sub_steps"], o
    for o in ("learned", "psi"):
        assert res[o][0] < res["none"][0], (o, res[o][0], res["none"][0])


def test_ktrace_load_kernel():
    """The k-trace reduction against numpy on a small trace with dead
    entries, a column never live and a ragged count."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2102_10983_amd import picsub
    rng = np.random.default_rng(7)
    steps, count = 37, 1000 + 13
    kt = rng.integers(-1, 6, size=(steps, count)).astype(np.int8)
    kt[:, 5] = -1
    got = picsub.ktrace_load(torch.from_numpy(kt).cuda()).cpu().numpy()
    live = kt >= 0
    tot = np.where(live, 4.0 ** np.maximum(kt, 0), 0.0).sum(0)
    n = live.sum(0)
    with np.errstate(divide="ignore", invalid="ignore"):
        want = np.log2(tot / n).astype(np.float32)
    assert np.isnan(got[5]) and np.isnan(want[5])
    ok = n > 0
    np.testing.assert_allclose(got[ok], want[ok], rtol=0, atol=2e-6)

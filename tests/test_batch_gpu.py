"""GPU tests of batches of uneven runs, device-driven windows, captured
graphs, the autotuner and the group dispatch order.

None of these may change a result: every run of a batch must equal the
same run pushed alone and the FP64 oracle, bit for bit in PIC_FP64.
"""

import sys

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


def _small_batch(seed=7, nruns=5, precision="fp64"):
    """Runs of different size, a0, dt and grid; one empty run."""
    runs = W.batch_case(seed=seed, nruns=nruns, periods=3.0, p_range=(50, 3000),
                        a0_range=(5.0, 150.0), cells_range=(400, 900))
    runs[2] = W.make_workload("empty", 0, 20.0, 40, 300, 3.0, 3, 0.01, 1.0, seed=99)
    return runs


def _state(d):
    return {k: d[k].copy() for k in ("x", "px", "py", "pz", "k_last", "status")}


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


def test_batch_equals_single_runs_and_oracle(torch_gpu):
    from paper_2102_10983_amd import runner
    from parity import compare
    wls = _small_batch()
    br = runner.BatchRun(wls, S=37, precision="fp64")
    br.reset()
    br.run_all()
    d = br.diag()
    per_run = [br.pusher.run_counters(r) for r in range(len(wls))]
    offs = br.pusher.offsets
    br.close()
    for r, wl in enumerate(wls):
        _say(f"run {r}: {wl.name} num={wl.num} steps={wl.steps}")
        sl = slice(offs[r], offs[r + 1])
        if wl.num == 0:
            assert per_run[r]["steps"] == 0
            continue
        one = runner.DeviceRun(wl, S=wl.steps, binning="none", precision="fp64")
        one.reset()
        one.advance(wl.steps)
        d1 = one.diag()
        one.close()
        for k in ("x", "px", "py", "pz", "k_last", "status"):
            assert np.array_equal(d[k][sl], d1[k]), (r, k)
        sub = {k: d[k][sl] for k in ("x", "px", "py", "pz", "status")}
        res = compare(wl, wl.steps, sub, np.arange(wl.num), 1e-12)
        assert res["bitwise"] == wl.num
        c = res["oracle_counters"]
        assert per_run[r]["steps"] == c.steps and per_run[r]["sub_steps"] == c.sub_steps


def test_graph_replays_match_eager(torch_gpu):
    """A captured pass replayed several times, with eager work between the
    replays, equals the eager pass every time."""
    torch = torch_gpu
    from paper_2102_10983_amd import runner
    wls = _small_batch(seed=8)
    eager = runner.BatchRun(wls, S=29, precision="fp64fast")
    eager.reset()
    eager.run_all()
    ref = _state(eager.diag())
    ref_cnt = eager.pusher.counters()
    eager.close()
    g = runner.BatchRun(wls, S=29, precision="fp64fast")
    g.reset()
    g.capture()
    for rep in range(3):
        g.reset()
        g.pusher.counters_reset()
        g.replay()
        torch.cuda.synchronize()
        got = g.diag()                         # eager copies between replays
        _ = torch.ones(1000, device="cuda").sum().item()
        assert _same(_state(got), ref), rep
        assert got["counters"] == ref_cnt, rep
        for r, wl in enumerate(wls):
            assert g.pusher.run_level(r) >= wl.steps
    g.pusher.graph_release()
    g.close()


@pytest.mark.parametrize("nbuckets", [1, 4])
def test_rebinning_between_graph_replays(torch_gpu, nbuckets):
    """Re-binning by a load score (group order only, or re-sorted slots)
    between replays of a captured pass: every replay equals the eager pass
    bit for bit (the graph's launches read the order and the particles from
    the arrays re-binning rewrites in place)."""
    torch = torch_gpu
    from paper_2102_10983_amd import runner
    wls = _small_batch(seed=8)
    eager = runner.BatchRun(wls, S=29, precision="fp64fast")
    eager.reset()
    eager.run_all()
    ref = _state(eager.diag())
    ref_cnt = eager.pusher.counters()
    eager.close()
    g = runner.BatchRun(wls, S=29, precision="fp64fast")
    g.reset()
    g.capture()
    num = sum(w.num for w in wls)
    for rep in range(3):
        g.reset()
        g.pusher.counters_reset()
        score = torch.from_numpy(np.random.default_rng(rep).random(num).astype(np.float32)).cuda()
        g.pusher.prebin(score, nbuckets=nbuckets, width=0.25)
        g.replay()
        torch.cuda.synchronize()
        got = g.diag()
        assert _same(_state(got), ref), rep
        assert got["counters"] == ref_cnt, rep
    g.pusher.graph_release()
    g.close()


def test_autotune_leaves_no_trace_and_keeps_results(torch_gpu):
    from paper_2102_10983_amd import runner
    wls = _small_batch(seed=9)
    b = runner.BatchRun(wls, S=40, precision="fp64")
    b.reset()
    before = _state(b.diag())
    best, ms = b.pusher.autotune(steps=40, reps=1)
    _say("autotune", best, ms)
    after = _state(b.diag())
    assert _same(before, after)
    assert b.pusher.counters()["steps"] == 0
    assert b.pusher.run_level(0) == 0
    b.run_all()
    tuned = _state(b.diag())
    b.close()
    ref = runner.BatchRun(wls, S=40, precision="fp64")
    ref.reset()
    ref.run_all()
    assert _same(tuned, _state(ref.diag()))
    ref.close()


@pytest.mark.parametrize("tune", [dict(waves_per_group=2), dict(waves_per_group=4),
                                  dict(binning="ballot", tile=128),
                                  dict(binning="ballot", tile=512)])
def test_launch_shapes_and_dispatch_order_change_nothing(torch_gpu, tune):
    from paper_2102_10983_amd import runner
    wls = _small_batch(seed=10)
    ref = runner.BatchRun(wls, S=31, precision="fp64")
    ref.reset()
    ref.run_all()
    want = _state(ref.diag())
    ref.close()
    b = runner.BatchRun(wls, S=31, precision="fp64")
    b.pusher.tune_set(**tune)
    ng = b.pusher.group_count()
    b.pusher.order_set(np.random.default_rng(1).permutation(ng).astype(np.int32))
    b.reset()
    b.run_all()
    assert _same(_state(b.diag()), want)
    b.close()


def test_order_must_be_a_permutation(torch_gpu):
    from paper_2102_10983_amd import picsub, runner
    b = runner.BatchRun(_small_batch(seed=11), S=10)
    ng = b.pusher.group_count()
    with pytest.raises(picsub.PicError):
        b.pusher.order_set(np.zeros(ng, dtype=np.int32))
    b.close()


def test_checkpoint_resume_equals_uninterrupted_run(torch_gpu):
    """Export after half the steps, import into a fresh context, finish:
    the same bits as the run that was never stopped (FP64), counters
    included; a mismatched context is refused."""
    from paper_2102_10983_amd import picsub, runner
    wls = _small_batch(seed=13)
    full = runner.BatchRun(wls, S=40, precision="fp64")
    full.reset()
    full.run_all()
    want = full.diag()
    full.close()

    a = runner.BatchRun(wls, S=40, precision="fp64")
    a.reset()
    a.pusher.advance(40)
    a.pusher.advance(40)
    blob = a.pusher.state_export()
    a.close()
    b = runner.BatchRun(wls, S=40, precision="fp64")
    b.pusher.particles_set(b.x0, *b.p0)
    lev = b.pusher.state_import(blob)
    assert all(lv == min(80, wl.steps) for lv, wl in zip(lev, wls))
    for r, (wl, (tab, M, co)) in enumerate(zip(b.wls, b.tables)):
        b.pusher.source_set(r, int(lev[r]), tab, M, co, n_stop=wl.steps)
    for _ in range(b.windows - 2):
        b.pusher.advance(40)
    got = b.diag()
    b.close()
    assert _same(_state(got), _state(want))
    assert got["counters"] == want["counters"]

    other = runner.BatchRun(_small_batch(seed=14), S=40, precision="fp64")
    other.reset()
    with pytest.raises(picsub.PicError):
        other.pusher.state_import(blob)
    other.close()


def test_diagnostics_in_a_captured_graph(torch_gpu):
    """Trajectory diagnostics switched on before the capture run inside the
    graph: replays give the eager values bit for bit (FP64); a captured
    graph keeps its setting when the diagnostics are switched off later."""
    from paper_2102_10983_amd import runner
    wls = _small_batch(seed=12)
    eager = runner.BatchRun(wls, S=29, precision="fp64", binning="none")
    eager.reset()
    eager.pusher.diag_track(True)
    eager.run_all()
    want_d = eager.pusher.dephasing_read()
    want_w = eager.pusher.energy_read()
    eager.close()
    g = runner.BatchRun(wls, S=29, precision="fp64", binning="none")
    g.reset()
    g.pusher.diag_track(True)
    g.capture()
    for rep in range(2):
        g.reset()                                  # tracking on: restarts the diagnostics
        g.replay()
        got_d = g.pusher.dephasing_read()
        got_w = g.pusher.energy_read()
        for a, b in zip(got_d + got_w, want_d + want_w):
            assert np.array_equal(a, b), rep
    g.pusher.diag_track(False)
    g.reset()                                      # loading particles restarts them (off too)
    assert not g.pusher.energy_read()[0].any()
    g.replay()                                     # the graph still updates them
    for a, b in zip(g.pusher.dephasing_read() + g.pusher.energy_read(), want_d + want_w):
        assert np.array_equal(a, b)
    g.pusher.graph_release()
    g.close()


def test_autotune_remembers_a_signature(torch_gpu):
    """A second context of the same configuration gets the first one's
    winner without trials (same time reported, no state touched); after
    pic_autotune_forget it is timed again."""
    import time
    from paper_2102_10983_amd import picsub, runner
    picsub.autotune_forget()
    wls = _small_batch(seed=15)
    a = runner.BatchRun(wls, S=40, precision="fp64fast")
    a.reset()
    best_a, ms_a = a.pusher.autotune(steps=40, reps=1)
    a.close()
    b = runner.BatchRun(wls, S=40, precision="fp64fast")
    b.reset()
    t0 = time.perf_counter()
    best_b, ms_b = b.pusher.autotune(steps=40, reps=1)
    cached_s = time.perf_counter() - t0
    assert best_b == best_a and ms_b == ms_a
    assert b.pusher.tune_get() == best_a
    assert b.pusher.counters()["steps"] == 0
    picsub.autotune_forget()
    _, ms_c = b.pusher.autotune(steps=40, reps=1)
    b.close()
    _say(f"cached lookup {cached_s * 1e3:.2f} ms, tuned {ms_a:.3f} / {ms_c:.3f} ms per window")
    assert ms_c != ms_a

"""The paper's model problem on the GPU (Sec. II): an electron at rest hit by
the Gaussian pulse, on a grid that moves with it between launches
(pic_grid_shift), against the FP64 oracle run over the same grids.  The
IEEE path is bit-identical to it (state, dephasing error of Eq. (R error),
counters); the fast path is within the metric's 1e-5 (k-flip protocol)
where the trajectory is well conditioned and matches the paper's trajectory
statistics where it amplifies rounding; and
the GPU runs reproduce the paper's printed claims that the oracle pins
(tests/test_pulse_oracle.py)."""

import sys

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W
from pulse_ref import run_whole, run_windows

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


def _gpu(torch, wl, precision, trace_steps=0):
    from paper_2102_10983_amd import runner
    run = runner.PulseRun(wl, S=1000, precision=precision)
    run.reset()
    buf = None
    if trace_steps:
        buf = torch.full((trace_steps, wl.num), -2, dtype=torch.int8, device="cuda")
        run.pusher.ktrace_set(buf, 0, 0)
    run.run(max_steps=trace_steps or (1 << 31))
    res = run.results()
    run.close()
    if buf is not None:
        res["ktrace"] = buf[:res["steps"]].cpu().numpy()
    return res


@pytest.mark.parametrize("a0", [25.0, 100.0])
def test_pulse_ieee_is_bit_identical_on_moving_grids(torch_gpu, a0):
    wl = W.pulse_case(a0, 75, 3, 0.01)
    _say(f"pulse IEEE a0={a0}")
    res = _gpu(torch_gpu, wl, "fp64")
    st, cnt, rmax, _, _, gmax = run_windows(wl, res["windows"], gamma_max=True)
    d = res["diag"]
    shifts = [w[2] for w in res["windows"]]
    _say(f"  {res['steps']} steps in {len(shifts)} launches, grid moved {shifts[-1]} cells, "
         f"eps_dephasing {rmax[0]:.4g}, N* {cnt.n_star}")
    for key, ref in (("x", st.x), ("px", st.px), ("py", st.py), ("pz", st.pz)):
        assert np.array_equal(d[key], ref), key
    assert np.array_equal(res["eps_dephasing"], rmax)
    assert np.array_equal(res["gamma_max"], gmax)
    c = d["counters"]
    assert (c["steps"], c["sub_steps"], c["n_star"]) == (cnt.steps, cnt.sub_steps, cnt.n_star)
    assert shifts[-1] > 10 * wl.ncells and rmax[0] < 0.1


def test_pulse_fast_path_within_tolerance(torch_gpu):
    """The benchmark arithmetic (FP64 with refined estimates) on the pulse at
    a0 = 5, where the trajectory is well conditioned: p and x within 1e-5 of
    the oracle over the same grids, the same decisions or a first flip at a
    threshold, epsilon_dephasing below 0.1."""
    wl = W.pulse_case(5.0, 75, 3, 0.01)
    _say("pulse fast a0=5")
    res = _gpu(torch_gpu, wl, "fp64fast", trace_steps=2_000_000)
    gk = res["ktrace"]
    st, cnt, rmax, kt, pt = run_windows(wl, res["windows"])
    flips = np.nonzero(np.any(gk != kt, axis=0))[0]
    if len(flips):
        s0 = int(np.argmax(gk[:, 0] != kt[:, 0]))
        kk = max(int(gk[s0, 0]), int(kt[s0, 0]))
        assert abs(pt[s0, 0] / 4.0 ** (kk - 1) - 1) < 1e-9
        st, cnt, rmax, _, _ = run_windows(wl, res["windows"], forced_k=gk)
    d = res["diag"]
    dp = np.sqrt((d["px"] - st.px) ** 2 + (d["py"] - st.py) ** 2 + (d["pz"] - st.pz) ** 2)
    e_p = dp / np.maximum(np.sqrt(st.px ** 2 + st.py ** 2 + st.pz ** 2), 1.0)
    e_x = np.abs(d["x"] - st.x) / np.maximum(np.abs(st.x - wl.x0), 2 * np.pi)
    _say(f"  {res['steps']} steps, flips {len(flips)}, e_p {e_p.max():.3g}, e_x {e_x.max():.3g}, "
         f"eps_dephasing {res['eps_dephasing'][0]:.4g} (oracle {rmax[0]:.4g})")
    assert e_p.max() <= 1e-5 and e_x.max() <= 1e-5
    assert res["eps_dephasing"][0] < 0.1


@pytest.mark.parametrize("a0", [25.0, 50.0, 100.0])
def test_pulse_fast_path_statistics(torch_gpu, a0):
    """At a0 >= 25 the pulse trajectory amplifies rounding (two oracle runs
    whose grid coordinates round differently end with momenta 3% apart at
    a0 = 25 and O(1) apart at a0 >= 50; tests/test_pulse_oracle.py), so the
    fast path is held to the trajectory statistics the paper reports rather
    than to the final state: epsilon_dephasing below 0.1 (Sec. VI) as for the
    oracle, the steps to clear the pulse and N* within 5% of the oracle's.
    The oracle runs on its own grid (not over the launches of the device
    run: a trajectory that has drifted from the device's leaves the device's
    moving grid); its own N* moves by ~3% between runs whose grid coordinates
    round differently (111,608 / 113,276 at a0 = 50, 172,212 / 177,416 at
    a0 = 100)."""
    wl = W.pulse_case(a0, 75, 3, 0.01)
    _say(f"pulse fast statistics a0={a0}")
    res = _gpu(torch_gpu, wl, "fp64fast")
    st, cnt, rmax, _ = run_whole(wl, chunk=1000)
    c = res["diag"]["counters"]
    _say(f"  {res['steps']} steps (oracle {cnt.steps}), N* {c['n_star']} (oracle {cnt.n_star}), "
         f"eps_dephasing {res['eps_dephasing'][0]:.4g} (oracle {rmax[0]:.4g})")
    assert res["eps_dephasing"][0] < 0.1 and rmax[0] < 0.1
    assert abs(c["n_star"] - cnt.n_star) < 0.05 * cnt.n_star
    assert abs(c["steps"] - cnt.steps) < 0.05 * cnt.steps


def test_pulse_claims_on_gpu(torch_gpu):
    """The paper's step-count and energy claims from GPU runs: N* about 20x
    for psi_max 0.01 -> 0.001 (a0 = 50, dt = lambda / 150 c, 1st order;
    Sec. V) and the 1st-order peak gamma about a third of the analytic one at
    a0 = 100 (Sec. IV; the running maximum after every step).  The bound is
    the oracle pin's: this 1st-order run amplifies rounding like the others
    (the oracle's own peak is 0.34 of the analytic one without sub-cycling
    and 0.26 with it; the fast path's run gives 0.22)."""
    n1 = _gpu(torch_gpu, W.pulse_case(50.0, 150, 1, 0.01), "fp64fast")["diag"]["counters"]["n_star"]
    n2 = _gpu(torch_gpu, W.pulse_case(50.0, 150, 1, 0.001), "fp64fast")["diag"]["counters"]["n_star"]
    g = _gpu(torch_gpu, W.pulse_case(100.0, 75, 1, 1e30), "fp64fast")["gamma_max"][0]
    ratio = g / (1.0 + 100.0 ** 2 / 2)
    _say(f"N* {n1} -> {n2} (x{n2 / n1:.1f}); 1st-order peak gamma / analytic {ratio:.3f}")
    assert 14 < n2 / n1 < 28 and 5e4 < n1 < 1e5
    assert 0.2 < ratio < 0.45


def test_second_order_accumulates_on_gpu(torch_gpu):
    """Sec. VI (Fig. 3b; a0 = 50, dt = lambda / 150 c, 2nd order, sub-cycling)
    on the GPU: the IEEE path on moving grids is bit-identical to the oracle
    over the same grids, and its dephasing error accumulates over the run
    (R / R_th - 1 ends negative, at about its largest magnitude) and stays
    far above the 3rd-order error (pinned on the CPU in
    tests/test_pulse_oracle.py)."""
    from oracle import oracle as O
    wl = W.pulse_case(50.0, 150, 2, 0.01)
    _say("pulse IEEE 2nd order a0=50 T/dt=150")
    res = _gpu(torch_gpu, wl, "fp64")
    st, cnt, rmax, _, _, gmax = run_windows(wl, res["windows"], gamma_max=True)
    d = res["diag"]
    for key, ref in (("x", st.x), ("px", st.px), ("py", st.py), ("pz", st.pz)):
        assert np.array_equal(d[key], ref), key
    assert np.array_equal(res["eps_dephasing"], rmax)
    assert np.array_equal(res["gamma_max"], gmax)
    eps = float(rmax[0])
    final = float(O.dephasing_R(d["px"], d["py"], d["pz"])[0] - 1.0)
    _say(f"  {res['steps']} steps, eps_dephasing {eps:.4g}, final R - 1 {final:+.4g}, "
         f"N* {d['counters']['n_star']}")
    assert final < 0 and abs(final) > 0.5 * eps and eps > 0.1

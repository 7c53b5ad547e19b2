"""GPU tests of the trajectory diagnostics kept by every push kernel when
switched on: the running maximum of |R - R0| / R0, R = gamma - p_x (Sec. V,
Eq. (R error)), and the energy accounting of App. B (work of E per
sub-step, largest single-step |d gamma - work|).

* PIC_FP64 (wavefront and ballot kernels, one launch and chunks of 16):
  all four arrays bit-identical to the FP64 oracle stepping one step at a
  time (oracle.push_diagnostics).
* PIC_FP64_FAST: within the bounds the 1e-5 bar on p implies,
  |d(R / R0)| <= 2e-5 max|p| / R0 and |d work|, |d err| <= 4e-5 max|p|, on
  electrons whose k sequence matches the oracle's (others are replayed
  with the device's k).
* Switching off freezes the values; re-binning carries them with the
  particles; loading particles restarts them.
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


def _gpu(torch, wl, S, precision, binning, fields="lattice"):
    from paper_2102_10983_amd import runner
    run = runner.DeviceRun(wl, S=S, precision=precision, binning=binning, fields=fields)
    run.reset()
    run.pusher.diag_track(True)
    buf = torch.full((wl.steps, wl.num), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, 0)
    run.advance(wl.steps)
    R0, rmax = run.pusher.dephasing_read()
    work, werr = run.pusher.energy_read()
    d = run.diag()
    d["work"], d["werr"] = work, werr
    d["gmax"] = run.pusher.gamma_max_read()
    kt = buf.cpu().numpy()
    run.close()
    return R0, rmax, d, kt


def _oracle(wl, fields=None, forced_k=None, idx=None):
    from oracle import oracle as O
    from parity import oracle_fields, oracle_params
    idx = np.arange(wl.num) if idx is None else idx
    st = O.State(wl.x0[idx], wl.p0[0][idx], wl.p0[1][idx], wl.p0[2][idx])
    fs = oracle_fields(wl) if fields is None else fields
    gmax = np.sqrt(1.0 + ((st.px * st.px + st.py * st.py) + st.pz * st.pz))
    R0, rmax, work, werr, kt = O.push_diagnostics(oracle_params(wl), fs, st, 0, wl.steps,
                                                   forced_k=forced_k, gmax=gmax)
    st.work, st.werr, st.gmax = work, werr, gmax
    return R0, rmax, kt, st


@pytest.mark.parametrize("S,binning", [(1500, "none"), (16, "none"), (16, "ballot")])
def test_fp64_bitwise(torch_gpu, S, binning):
    wl = W.small_case(order=3)
    _say(f"dephasing fp64 S={S} binning={binning}")
    R0, rmax, d, kt = _gpu(torch_gpu, wl, S, "fp64", binning)
    oR0, ormax, okt, st = _oracle(wl)
    assert np.array_equal(kt, okt)
    assert np.array_equal(R0, oR0)
    assert np.array_equal(rmax, ormax)
    assert np.array_equal(d["px"], st.px)
    assert np.array_equal(d["work"], st.work) and np.array_equal(d["werr"], st.werr)
    assert np.array_equal(d["gmax"], st.gmax) and np.all(d["gmax"] >= d["gamma"])
    _say("max eps_dephasing", float(rmax.max()), "max step energy error", float(d["werr"].max()))
    assert rmax.max() > 0 and d["werr"].max() > 0 and d["work"].max() > 1.0


def test_fp64_bitwise_with_losses_and_standard_pic(torch_gpu):
    """Thermal electrons (R0 != 1), some leaving the grid, on Yee levels."""
    from parity import oracle_yee_fields
    wl = W.make_workload("th", 2000, 60.0, 75, 400, 3, 3, 0.01, 3.0, seed=43,
                         theta=10.0 / 511.0)
    R0, rmax, d, kt = _gpu(torch_gpu, wl, 50, "fp64", "none", fields="yee")
    oR0, ormax, okt, st = _oracle(wl, fields=oracle_yee_fields(wl, wl.steps))
    assert d["counters"]["lost"] > 0
    assert np.array_equal(kt, okt)
    assert np.array_equal(R0, oR0) and np.array_equal(rmax, ormax)
    assert np.array_equal(d["work"], st.work) and np.array_equal(d["werr"], st.werr)
    assert np.array_equal(d["gmax"], st.gmax)
    assert np.ptp(R0) > 0.01


@pytest.mark.parametrize("a0,theta", [(10.0, 0.0), (100.0, 10.0 / 511.0)])
def test_fp64fast_within_the_implied_bound(torch_gpu, a0, theta):
    wl = W.make_workload("f", 1024, a0, 75, 1200, 6, 3, 0.01, 2.0, seed=44, theta=theta)
    R0, rmax, d, kt = _gpu(torch_gpu, wl, wl.steps, "fp64fast", "none")
    oR0, ormax, okt, st = _oracle(wl)
    same = np.all(kt == okt, axis=0)
    owork, owerr, ogmax = st.work.copy(), st.werr.copy(), st.gmax.copy()
    if not same.all():
        idx = np.nonzero(~same)[0]
        _, fr, _, fst = _oracle(wl, forced_k=np.ascontiguousarray(kt[:, idx]), idx=idx)
        ormax = ormax.copy()
        ormax[idx] = fr
        owork[idx], owerr[idx], ogmax[idx] = fst.work, fst.werr, fst.gmax
    pmax = a0 * a0 / 2 + a0 + 1.0               # bound on |p| along a plane-wave orbit
    bound = 2 * 1e-5 * pmax / oR0
    err = np.abs(rmax - ormax)
    ew = np.abs(d["work"] - owork)
    ee = np.abs(d["werr"] - owerr)
    _say(f"a0={a0}: flips {int((~same).sum())}, max |d rmax| {err.max():.3e}, "
         f"largest allowed {bound.min():.3e}; max |d work| {ew.max():.3e}, "
         f"max |d err| {ee.max():.3e}, allowed {4e-5 * pmax:.3e}")
    assert np.all(err <= bound)
    assert np.all(ew <= 4e-5 * pmax) and np.all(ee <= 4e-5 * pmax)
    assert np.all(np.abs(d["gmax"] - ogmax) <= 2e-5 * pmax)    # |d gamma| <= |d p|
    assert np.allclose(R0, oR0, rtol=1e-12, atol=0)


def test_off_freezes_prebin_carries_load_restarts(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import runner
    wl = W.small_case(order=3, num=1024, periods=4)
    half = wl.steps // 2

    def run_once(rebin):
        run = runner.DeviceRun(wl, S=wl.steps, precision="fp64", binning="none")
        run.reset()
        run.pusher.diag_track(True)
        run.advance(half)
        if rebin:      # a score that reverses positions moves every particle
            score = torch.from_numpy(-wl.x0.astype(np.float32)).cuda()
            run.pusher.prebin(score, nbuckets=8, width=0.5)
        run.advance(wl.steps - half)
        return run

    ref = run_once(False)
    _, m_ref = ref.pusher.dephasing_read()
    w_ref = ref.pusher.energy_read()
    g_ref = ref.pusher.gamma_max_read()
    ref.close()
    run = run_once(True)
    R0, m = run.pusher.dephasing_read()
    assert np.array_equal(m, m_ref) and np.all(R0 == 1.0) and m.max() > 0
    w = run.pusher.energy_read()
    assert np.array_equal(w[0], w_ref[0]) and np.array_equal(w[1], w_ref[1])
    assert np.array_equal(run.pusher.gamma_max_read(), g_ref) and g_ref.max() > 1.0
    run.pusher.diag_track(False)              # off: later steps change nothing
    run.advance(40)
    _, m_off = run.pusher.dephasing_read()
    assert np.array_equal(m_off, m)
    run.pusher.diag_track(True)               # on again: restarts from the state now
    R0b, m0 = run.pusher.dephasing_read()
    assert np.all(m0 == 0.0) and not np.all(R0b == 1.0)
    d = run.diag()
    live = d["status"] == 0
    assert np.allclose(run.pusher.gamma_max_read()[live], d["gamma"][live], rtol=1e-15, atol=0)
    run.advance(20)
    assert run.pusher.dephasing_read()[1].max() > 0
    run.reset()                                    # loading particles restarts it
    R0c, mc = run.pusher.dephasing_read()
    assert np.all(mc == 0.0) and np.all(R0c == 1.0)
    assert not run.pusher.energy_read()[0].any()
    run.close()

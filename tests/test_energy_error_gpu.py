"""The energy error of Sec. IV, Eq. (gamma error), computed by the push
kernels on the GPU: the running maximum of |gamma - gamma_th| / gamma_th
against the plane-wave solution gamma_th = 1 + (a - a_i)^2 / 2
(Eq. (theoretical gamma)), a at the phase of the momentum.

Electrons at rest in the Gaussian pulse of the paper's model problem
(Sec. II) on a grid that moves with them, against the FP64 oracle over the
same grids: the IEEE kernels (wavefronts and ballot compaction) give the
oracle's maxima bit for bit, also across a re-binning between launches; the
fast and FP32-compensated kernels stay within the bounds their accuracy
on the state implies, on a well-conditioned trajectory; and the GPU runs reproduce the growth of the
1st-order error with a0 that the paper reports (Fig. 2b), which the oracle
pins in tests/test_pulse_oracle.py."""

import dataclasses
import sys

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W
from pulse_ref import run_windows

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


def _spread(wl, num, width):
    """The pulse workload with num electrons at rest over [0, width)."""
    x0 = np.linspace(0.0, width, num, endpoint=False)
    return dataclasses.replace(wl, num=num, x0=x0, p0=np.zeros((3, num)))


def _run(wl, precision, S=1000, binning=None, rebin_after_first=False, seed=0):
    from paper_2102_10983_amd import runner
    import torch
    run = runner.PulseRun(wl, S=S, precision=precision, energy=True)
    if binning:
        run.pusher.tune_set(binning=binning)
    run.reset()
    first = True
    while run.window():
        if first and rebin_after_first:
            # a random group order and slot layout; results must not change
            g = torch.Generator().manual_seed(seed)
            score = torch.rand(wl.num, generator=g).to("cuda")
            run.pusher.prebin(score, nbuckets=4, width=0.25)
        first = False
    res = run.results()
    run.close()
    return res


@pytest.mark.parametrize("binning,rebin", [(None, False), (None, True), ("ballot", False)])
def test_energy_error_ieee_bitwise(torch_gpu, binning, rebin):
    wl = _spread(W.pulse_case(5.0, 75, 3, 0.01), 200, 0.5 * np.pi)
    _say(f"energy error IEEE binning={binning} rebin={rebin}")
    res = _run(wl, "fp64", S=500, binning=binning, rebin_after_first=rebin)
    st, cnt, rmax, _, _, gmax, emax = run_windows(wl, res["windows"], gamma_max=True,
                                                  energy=True)
    d = res["diag"]
    _say(f"  {res['steps']} steps in {len(res['windows'])} launches, eps_energy "
         f"{emax.min():.4g} .. {emax.max():.4g}")
    for key, ref in (("x", st.x), ("px", st.px), ("py", st.py), ("pz", st.pz)):
        assert np.array_equal(d[key], ref), key
    assert np.array_equal(res["eps_dephasing"], rmax)
    assert np.array_equal(res["gamma_max"], gmax)
    assert np.array_equal(res["eps_energy"], emax)
    assert emax.max() > 0 and emax.max() < 0.05


@pytest.mark.parametrize("precision,tol", [("fp64fast", 1e-6), ("fp32c", 1e-3)])
def test_energy_error_fast_paths(torch_gpu, precision, tol):
    """The maxima against the oracle's over the same grids.  The bound
    follows from each path's accuracy on the state: the fast path's p and x
    errors stay below 1e-6 here; the FP32-compensated path's x is held to 1e-5
    of the distance travelled (about 1e3 c / omega in this run), which moves
    the phase where gamma_th is taken, and a = a0 sin(phase) moves gamma_th by
    up to a0 |a - a_i| 1e-2 relative to it (measured: 1.5e-4 on the worst of
    200 electrons, 1e-7 on the median)."""
    wl = _spread(W.pulse_case(5.0, 75, 3, 0.01), 200, 0.5 * np.pi)
    _say(f"energy error {precision}")
    res = _run(wl, precision, S=500)
    emax = run_windows(wl, res["windows"], energy=True)[-1]
    err = np.abs(res["eps_energy"] - emax)
    _say(f"  eps_energy {emax.max():.4g}, largest difference {err.max():.3g}, "
         f"median {np.median(err):.3g}")
    assert err.max() < tol


def test_energy_error_start_and_errors(torch_gpu):
    from paper_2102_10983_amd import picsub
    wl = W.pulse_case(5.0, 75, 3, 0.01)
    table, M, shift = wl.table()
    p = picsub.Pusher(num=4, ncells=wl.ncells, order=3, dx=wl.dx, dt=wl.dt, psi_max=0.01,
                      x_origin=wl.x_origin, ring_depth=16, precision="fp64", binning="none")
    try:
        p.particles_set(np.zeros(4), np.zeros(4), np.zeros(4), np.zeros(4))
        atab = torch_gpu.from_numpy(np.ascontiguousarray(wl.potential()[0])).cuda()
        with pytest.raises(picsub.PicError) as e:
            p.gamma_error_start(np.zeros(4))               # diagnostics off
        assert e.value.status == 5
        p.diag_track(True)
        with pytest.raises(picsub.PicError) as e:
            p.gamma_error_read()                          # not started
        assert e.value.status == 1
        with pytest.raises(picsub.PicError) as e:
            p.gamma_error_lattice(atab, 0, (1, 1, 0))     # empty lattice
        assert e.value.status == 1
        with pytest.raises(picsub.PicError) as e:
            p.gamma_error_lattice(atab, M, (1, 1, 0), run=3)
        assert e.value.status == 1
        with pytest.raises(ValueError):
            p.gamma_error_start(np.zeros(3))
        p.gamma_error_start(np.zeros(4))
        assert np.array_equal(p.gamma_error_read(), np.zeros(4))
        p.particles_set(np.zeros(4), np.zeros(4), np.zeros(4), np.zeros(4))
        with pytest.raises(picsub.PicError):
            p.gamma_error_read()                          # new particles: stopped
        p.gamma_error_lattice(None, 0, (0, 0, 0))         # detach
    finally:
        p.close()


def test_first_order_energy_error_grows_with_a0_on_gpu(torch_gpu):
    """Sec. IV (Fig. 2b) from GPU runs (benchmark arithmetic): with 1st-order
    interpolation and no sub-cycling at dt = lambda / 75 c the energy error
    grows with a0 and is significant beyond a0 ~ 40; 3rd order with
    sub-cycling keeps it an order of magnitude lower there.  The bounds are
    the oracle pin's (its values: 0.02, 0.07, 0.40, 1.7, 9.8 against 0.003,
    0.005, 0.05, 0.06, 0.19 at a0 = 5, 10, 25, 50, 100) except at a0 = 25,
    below the range of the claim, where the pin's 5x margin becomes 2x: that
    trajectory amplifies rounding (the fast path's run gives 0.078 against
    0.39; GPU values 0.020, 0.069, 0.39, 1.5, 5.2 and 0.0027, 0.0053, 0.078,
    0.064, 0.13)."""
    e1, e3 = [], []
    for a0 in (5.0, 10.0, 25.0, 50.0, 100.0):
        e1.append(float(_run(W.pulse_case(a0, 75, 1, 1e30), "fp64fast")["eps_energy"][0]))
        e3.append(float(_run(W.pulse_case(a0, 75, 3, 0.01), "fp64fast")["eps_energy"][0]))
    _say(f"1st order {['%.3g' % v for v in e1]}, 3rd order with sub-cycling "
         f"{['%.3g' % v for v in e3]}")
    assert all(a < b for a, b in zip(e1, e1[1:])), e1
    assert e1[0] < 0.05 and min(e1[3:]) > 1.0, e1
    assert e3[2] < 0.5 * e1[2], (e1, e3)
    assert all(b < 0.1 * a for a, b in zip(e1[3:], e3[3:])), (e1, e3)

"""Paper-level pins of the oracle on the model problem of Sec. II: one
electron at rest hit by the Gaussian pulse (xi0 = 160 pi after the
electron's initial phase, sigma = 8 pi), prescribed fields ("perfectly
propagating PIC"), c dt / dx = 1 / 1.01.  Each test checks a number or a
trend the paper prints, with a loose bound: the paper's figure data are not
available, its own runs differ in details it does not state, and the
quantities are maxima along a trajectory.

Not pinned (measured here, recorded in the design notes): the location of
the maximum of chi^3 (the paper finds a0 ~ 25 at T/dt = 75; here the ratio
is noisy and largest near a0 = 75), the absence of a rollover of chi^5 at
a0 <= 100 (here chi^5 is as noisy: 47, 39, 139, 104, 86, 157 at a0 = 5, 10,
25, 50, 75, 100) and a stopping point at t omega ~ 9110 for a0 = 50,
T/dt = 150 (here the nearest are at 8585 and 9483).
"""

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W
from pulse_ref import run_whole


def _run(a0, n_t, order, psi):
    return run_whole(W.pulse_case(a0, n_t, order, psi))


def _run_nt(a0, n_t, order, psi):
    return run_whole(W.pulse_case(a0, n_t, order, psi), chunk=1000)


@pytest.mark.parametrize("a0", [5.0, 25.0, 50.0, 100.0])
def test_third_order_with_subcycling_keeps_dephasing_below_a_tenth(a0):
    """Sec. VI: with 3rd-order interpolation and sub-cycling (psi_max = 0.01)
    at dt = lambda / 75 c, epsilon_dephasing stays below 0.1 for every
    5 <= a0 <= 100; with 1st order it is far larger (Sec. IV)."""
    _, _, r3, _ = _run(a0, 75, 3, 0.01)
    _, _, r1, _ = _run(a0, 75, 1, 0.01)
    assert r3[0] < 0.1
    assert r1[0] > 10 * r3[0]          # "at least an order of magnitude" (Sec. I)


def test_first_order_underestimates_the_peak_energy_threefold():
    """Sec. IV: at a0 = 100 and dt = lambda / 75 c the 1st-order algorithm
    reaches about a third of the analytic peak gamma = 1 + a0^2 / 2, with or
    without sub-cycling; 3rd order with sub-cycling reaches it."""
    g_th = 1.0 + 100.0 ** 2 / 2
    for psi in (1e30, 0.01):
        _, _, _, g = _run(100.0, 75, 1, psi)
        assert 0.2 < g[0] / g_th < 0.45, (psi, g[0] / g_th)
    _, _, _, g3 = _run(100.0, 75, 3, 0.01)
    assert 0.9 < g3[0] / g_th < 1.1


def test_tighter_psi_max_multiplies_subcycled_steps_about_twentyfold():
    """Sec. V: at a0 = 50, dt = lambda / 150 c, 1st order, psi_max = 0.01
    -> 0.001 takes the sub-cycled steps N* from about 72,000 to about
    1.5e6, a factor of about 21."""
    _, c1, _, _ = _run(50.0, 150, 1, 0.01)
    _, c2, _, _ = _run(50.0, 150, 1, 0.001)
    assert 5e4 < c1.n_star < 1e5, c1.n_star
    assert 1e6 < c2.n_star < 2e6, c2.n_star
    assert 14 < c2.n_star / c1.n_star < 28


def test_subcycled_share_falls_as_a0_grows():
    """Sec. VI: delta_steps = N* / (N* + N) decreases with a0 (the travel
    time between stopping points grows), 3rd order, psi_max = 0.01,
    dt = lambda / 75 c."""
    ds = []
    for a0 in (10.0, 25.0, 50.0, 100.0):
        _, c, _, _ = _run(a0, 75, 3, 0.01)
        ds.append(c.n_star / (c.n_star + c.steps))
    assert all(a > b for a, b in zip(ds, ds[1:])), ds


@pytest.mark.parametrize("a0", [5.0, 25.0, 50.0, 100.0])
def test_standard_algorithm_needs_dt_lambda_over_600(a0):
    """Sec. VI: the standard algorithm (1st order, no sub-cycling) needs
    dt = lambda / 600 c to match the new algorithm at lambda / 75 c:
    epsilon_dephasing below 0.1 there for 5 <= a0 <= 100."""
    _, _, r, _ = _run(a0, 600, 1, 1e30)
    assert r[0] < 0.1


def test_long_pulse_runs_amplify_rounding():
    """Over the ~10^5 steps of a pulse at a0 = 25 the trajectory amplifies
    rounding: the oracle on one long grid and on grids that move with the
    electron (the same nodes, only the grid coordinate rounded differently)
    end with momenta a few percent apart, while the paper's trajectory
    statistics hold on both (epsilon_dephasing below 0.1, N* within a few
    percent).  At a0 >= 50 the final momenta differ by O(1) (measured: also
    for x0 moved by 1e-12), and epsilon_dephasing by up to a factor of two
    while staying below 0.1; arithmetic that is not bit-identical is compared
    on those statistics there."""
    from pulse_ref import moving_windows, run_windows
    wl = W.pulse_case(25.0, 75, 3, 0.01)
    sw, cw, rw, _, _ = run_windows(wl, moving_windows(wl))
    s1, c1, r1, _ = run_whole(wl, chunk=1000)
    dp = float(np.hypot(sw.px[0] - s1.px[0], sw.py[0] - s1.py[0]))
    e_p = dp / max(1.0, float(np.hypot(s1.px[0], s1.py[0])))
    assert e_p > 1e-3
    assert max(rw[0], r1[0]) < 0.1
    assert abs(cw.n_star - c1.n_star) < 0.05 * c1.n_star


def test_second_order_improves_marginally_and_accumulates():
    """Sec. VI (Fig. 3b; a0 = 50, dt = lambda / 150 c, with sub-cycling):
    2nd-order interpolation (two past levels, one future) improves on 1st
    order only marginally, where 3rd order improves dramatically, and its
    error accumulates over the run instead of returning towards zero after
    the pulse has overtaken the electron as the 1st-order error does;
    R / R_th - 1 ends negative."""
    from oracle import oracle as O
    out = {}
    for order in (1, 2, 3):
        st, _, r, _ = _run_nt(50.0, 150, order, 0.01)
        out[order] = (r[0], float(O.dephasing_R(st.px, st.py, st.pz)[0] - 1.0))
    (e1, f1), (e2, f2), (e3, _) = out[1], out[2], out[3]
    assert 0.4 * e1 < e2 < e1            # marginal
    assert e3 < 0.05 * e1                # dramatic
    assert abs(f1) < 0.2 * e1            # 1st order returns towards zero
    assert f2 < 0 and abs(f2) > 0.5 * e2  # 2nd order accumulates, downwards


@pytest.mark.parametrize("a0", [5.0, 25.0, 50.0, 100.0])
def test_fifth_order_keeps_the_step_count_and_the_accuracy(a0):
    """Sec. VII: with the same sub-cycling condition (psi_max = 0.01,
    dt = lambda / 75 c) delta_steps is mostly unaffected by going from 3rd
    to 5th order (the trajectories are very similar), and 5th order with
    sub-cycling is as accurate: epsilon_dephasing below 0.1 and at least an
    order of magnitude below 1st order."""
    d = {}
    for order in (1, 3, 5):
        _, c, r, _ = _run(a0, 75, order, 0.01)
        d[order] = (r[0], c.n_star / (c.n_star + c.steps))
    assert abs(d[5][1] - d[3][1]) < 0.15 * d[3][1]
    assert d[5][0] < 0.1 and d[1][0] > 10 * d[5][0]


def _energy_error_flat(n_t):
    """Largest energy error of 64 electrons at rest in a flat a0 = 1 wave over
    two periods, 1st order, no sub-cycling."""
    from oracle import oracle as O
    from pulse_ref import a_on_lattice
    wl = W.make_workload("e", 64, 1.0, n_t, 4 * n_t, 2.0, 1, 1e30, 1.0, seed=5)
    table, M, shift = wl.table()
    atab, _, _ = wl.potential()
    co = W.shifted_coeffs(wl.lat, shift)
    fs = O.FieldSource(table=table, M=M, coeffs=co, atab=atab)
    prm = O.make_params(wl.ncells, 1, wl.dx, wl.dt, wl.psi_max, wl.x_origin)
    st = O.State(wl.x0, *wl.p0)
    emax = np.zeros(wl.num)
    O.push(prm, fs, st, 0, wl.steps, ai=a_on_lattice(wl, atab, M, co, -0.5, wl.x0), emax=emax)
    return float(emax.max())


def test_energy_error_converges_at_second_order():
    """The energy error of Eq. (gamma error) against Eq. (theoretical gamma)
    on a flat wave falls 4x per halving of dt: the integrator is second order
    and gamma_th is taken at the phase of the momentum (half a sub-step
    behind x).  Taking it at the phase of x instead leaves an O(dt) error
    (first order, 30x larger at T/dt = 150), which this fails."""
    e = [_energy_error_flat(n) for n in (150, 300, 600)]
    assert e[0] < 1e-3
    for a, b in zip(e, e[1:]):
        assert 3.5 < a / b < 4.6, e


def test_first_order_energy_error_grows_with_a0():
    """Sec. IV (Fig. 2b): with 1st-order interpolation and no sub-cycling at
    dt = lambda / 75 c, epsilon_energy increases almost monotonically with
    a0 and becomes significant beyond a0 ~ 40; 3rd order with sub-cycling
    keeps it an order of magnitude lower there (measured: 0.02, 0.07, 0.40,
    1.7, 9.8 against 0.003, 0.005, 0.05, 0.06, 0.19 for a0 = 5, 10, 25, 50,
    100)."""
    e1, e3 = [], []
    for a0 in (5.0, 10.0, 25.0, 50.0, 100.0):
        e1.append(float(run_whole(W.pulse_case(a0, 75, 1, 1e30), chunk=1000, energy=True)[4][0]))
        e3.append(float(run_whole(W.pulse_case(a0, 75, 3, 0.01), chunk=1000, energy=True)[4][0]))
    assert all(a < b for a, b in zip(e1, e1[1:])), e1
    assert e1[0] < 0.05 and min(e1[3:]) > 1.0, e1
    assert e3[2] < 0.2 * e1[2], (e1, e3)
    assert all(b < 0.1 * a for a, b in zip(e1[3:], e3[3:])), (e1, e3)

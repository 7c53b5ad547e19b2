"""Host logic of the model-problem runs (no GPU): the a_i the product hands
the energy error equals the oracle side's, the end-of-run rule, the
closed-form duration that caps a run, and chi."""

import math

import numpy as np

from paper_2102_10983_amd import pulse_sweep as PS
from paper_2102_10983_amd import runner
from paper_2102_10983_amd import workloads as W
from pulse_ref import a_on_lattice


def test_initial_potential_is_the_oracle_sides():
    wl = W.pulse_case(25.0, 75, 3, 0.01, num=7)
    wl.x0[:] = np.linspace(0.0, 3.0, 7)
    table, M, shift = wl.table()
    atab, aM, ashift = wl.potential()
    assert (aM, ashift) == (M, shift)
    co = W.shifted_coeffs(wl.lat, shift)
    got = runner.initial_potential(wl, atab, M, co)
    want = a_on_lattice(wl, atab, M, co, -0.5, wl.x0)
    assert np.array_equal(got, want)
    # the pulse is far from the electrons at the start: a_i is (almost) zero
    assert np.all(np.abs(got) < 1e-6 * 25.0)


def test_pulse_passed_rule():
    wl = W.pulse_case(5.0, 75, 3, 0.01, num=2)
    xi_end = W.GAUSS_XI0 + 7.0 * W.GAUSS_SIGMA
    n = int(math.ceil((xi_end + 10.0) / wl.dt))
    x = np.array([0.0, 20.0])
    live = np.zeros(2, dtype=np.uint8)
    assert not runner.pulse_passed(wl, 10, x, live)             # the pulse has not arrived
    assert not runner.pulse_passed(wl, n, x, live)              # passed one, not the other
    assert runner.pulse_passed(wl, n, np.array([0.0, 9.0]), live)
    assert runner.pulse_passed(wl, n, x, np.array([0, 1], dtype=np.uint8))  # the other is lost
    assert runner.pulse_passed(wl, 10, x, np.ones(2, dtype=np.uint8))       # none live


def test_analytic_steps_is_the_closed_form():
    """t = xi_end + x with x = (1/2) int a^2 dxi; for a Gaussian envelope of
    width sigma and a fast sin, int a^2 = a0^2 sigma sqrt(pi) / 2.  Checked
    by quadrature of the pulse's own potential."""
    xi_end = W.GAUSS_XI0 + 7.0 * W.GAUSS_SIGMA
    assert PS.analytic_steps(0.0, 75) == math.ceil(xi_end / (2 * math.pi / 75))
    xi = np.linspace(W.GAUSS_XI0 - 10 * W.GAUSS_SIGMA, W.GAUSS_XI0 + 10 * W.GAUSS_SIGMA, 400001)
    a = np.exp(-(xi - W.GAUSS_XI0) ** 2 / (2 * W.GAUSS_SIGMA ** 2)) * np.sin(xi)
    x = 0.5 * np.trapezoid(a * a, xi)
    for a0, n_t in ((10.0, 75), (100.0, 600)):
        t = xi_end + a0 * a0 * x
        assert abs(PS.analytic_steps(a0, n_t) - t / (2 * math.pi / n_t)) < 1e-4 * t / (2 * math.pi / n_t) + 1


def test_chi_pairs_orders_with_subcycling_only():
    recs = [{"order": o, "n_t": 75, "a0": 5.0, "subcycling": sub, "eps_dephasing": e}
            for o, sub, e in ((1, True, 0.5), (3, True, 0.01), (5, True, 0.02), (1, False, 9.0),
                              (3, False, 1.0))]
    assert PS.chi(recs, 3) == {(75, 5.0): 50.0}
    assert PS.chi(recs, 5) == {(75, 5.0): 25.0}
    S, cells = PS.window_steps(600)
    assert S == 6000 and cells >= 8 + S * 100 // 101 + 16

"""Pins of the FP64 Yee reference (Sec. III, Eqs. (Ey) and (Bz)) against
facts that do not come from the reference itself:

* at dt = dx (the "magic" time step of the 1D Yee scheme) any right-going
  wave is carried exactly, bit for bit when its samples lie in [1, 2)
  (every difference is then exact), and the Mur condition reduces to
  exact transport;
* at the paper's dt = dx / 1.01 a right-going wave quadratic in x - t is
  an exact solution of the centred updates, of the Mur condition and of
  the source, so the grid must hold its samples to rounding;
* a sinusoid is carried with the textbook numerical dispersion of the
  Yee scheme, sin(w dt / 2) = (dt / dx) sin(k dx / 2), with equal E and B
  amplitudes, on every node the right boundary cannot yet have reached.
"""

import math

import numpy as np
import pytest

from oracle import yee_ref as Y


def _samples(f, n, ncells, dx, dt):
    """E at ((i + 1/2) dx, n dt), B at (i dx, (n + 1/2) dt)."""
    i = np.arange(ncells)
    return f((i + 0.5) * dx - n * dt), f(i * dx - (n + 0.5) * dt)


def test_magic_time_step_is_exact_transport():
    rng = np.random.default_rng(3)
    ncells, count = 97, 150
    T = 1.0 + rng.random(2 * (ncells + count) + 8)      # samples in [1, 2)
    off = 2 * count + 4

    def E_at(n):
        return T[2 * (np.arange(ncells) - n) + 1 + off]

    def B_at(n):                       # B at t = (n + 1/2) dt
        return T[2 * (np.arange(ncells) - n) - 1 + off]

    d = 0.0837
    b0 = [T[2 * (0 - m) - 1 + off] for m in range(1, count + 1)]
    El, Bl = Y.advance(E_at(0), B_at(0), d, d, b0)
    for c in range(count):
        assert np.array_equal(El[c], E_at(c + 1)), c
        assert np.array_equal(Bl[c], B_at(c + 1)), c


def test_quadratic_wave_is_exact_at_the_papers_courant_number():
    dt = 2 * math.pi / 75
    dx = 1.01 * dt
    ncells, count = 160, 300                      # the wave crosses the right end

    def f(u):
        return 0.7 - 0.3 * u + 0.02 * u * u

    E0, B0 = _samples(f, 0, ncells, dx, dt)
    b0 = [f(0.0 - (m + 0.5) * dt) for m in range(1, count + 1)]
    El, Bl = Y.advance(E0, B0, dx, dt, b0)
    scale = max(np.abs(El).max(), np.abs(Bl).max())
    for c in range(count):
        Ew, Bw = _samples(f, c + 1, ncells, dx, dt)
        assert np.abs(El[c] - Ew).max() < 1e-12 * scale, c
        assert np.abs(Bl[c] - Bw).max() < 1e-12 * scale, c


def test_mur_coefficient_and_courant_number():
    nu, kappa = Y.coefficients(1.01, 1.0)
    assert nu == 1.0 / 1.01
    assert kappa == (1.0 - 1.01) / (1.0 + 1.01)
    assert Y.coefficients(0.5, 0.5) == (1.0, 0.0)


@pytest.mark.parametrize("ppw", [75.0 / 1.01, 20.0])
def test_sinusoid_follows_the_yee_dispersion_relation(ppw):
    dt = 2 * math.pi / 75
    dx = 1.01 * dt
    nu = dt / dx
    k = 2 * math.pi / (ppw * dx)                  # ppw nodes per wavelength
    w = 2.0 / dt * math.asin(nu * math.sin(k * dx / 2))
    ncells, count = 600, 200

    def wave(omega):
        def f_xt(x, t):
            return np.sin(k * x - omega * t)
        return f_xt

    i = np.arange(ncells)

    def levels(omega, n):
        g = wave(omega)
        return g((i + 0.5) * dx, n * dt), g(i * dx, (n + 0.5) * dt)

    E0, B0 = levels(w, 0)
    b0 = [math.sin(-w * (m + 0.5) * dt) for m in range(1, count + 1)]
    El, Bl = Y.advance(E0, B0, dx, dt, b0)
    for c in range(count):
        reach = ncells - 1 - (c + 2)      # nodes the Mur boundary cannot have reached
        Ew, Bw = levels(w, c + 1)
        assert np.abs(El[c, :reach] - Ew[:reach]).max() < 1e-11, c
        assert np.abs(Bl[c, :reach] - Bw[:reach]).max() < 1e-11, c
    # the vacuum relation w = k is measurably wrong at this resolution
    Ev, _ = levels(k, count)
    assert np.abs(El[-1, :ncells - count - 3] - Ev[:ncells - count - 3]).max() > 1e-6


def test_outgoing_pulse_leaves_little_behind():
    """A Gaussian pulse that has left through the Mur boundary leaves a
    reflection far below its amplitude (first-order Mur is exact for waves
    up to quadratic in x - t; a 30-node pulse is close to that)."""
    dt = 2 * math.pi / 75
    dx = 1.01 * dt
    ncells = 300

    def f(u):
        return np.exp(-((u + 12.0) / 2.5) ** 2)

    E0, B0 = _samples(f, 0, ncells, dx, dt)
    count = 700
    b0 = [float(f(np.array(-(m + 0.5) * dt))) for m in range(1, count + 1)]
    El, Bl = Y.advance(E0, B0, dx, dt, b0)
    assert np.abs(El[150]).max() > 0.5            # pulse inside the grid
    assert np.abs(El[-1]).max() < 2e-3
    assert np.abs(Bl[-1]).max() < 2e-3


def test_lattice_source_indexing():
    table = np.arange(11, dtype=np.float64)
    E = np.zeros(5)
    B = np.zeros(5)
    _, Bl = Y.advance_lattice(E, B, 1.0, 0.5, -3, 4, table, aB=3, cB=2)
    assert list(Bl[:, 0]) == [table[(3 * m + 2) % 11] for m in range(-3, 1)]

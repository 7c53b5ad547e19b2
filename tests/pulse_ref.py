"""The FP64 oracle on the paper's model problem (Sec. II): electrons at rest
hit by the Gaussian pulse of workloads.pulse_case, sampled from the same
phase table the device uses.

Two ways to run it:
* whole: one grid long enough for the whole path (the oracle samples the
  table node by node, so a long grid costs nothing), until the pulse has
  passed (phase t - x beyond xi0 + 7 sigma), checked every `chunk` steps;
* windows: the grids of a device run that moved its grid with the
  electrons (runner.PulseRun.windows: start level, steps and shift of every
  launch), so that every step sees the same nodes as on the device.
"""

from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_2102_10983_amd import workloads as W

XI_END = W.GAUSS_XI0 + 7.0 * W.GAUSS_SIGMA


def _fields(wl, shift=0, atab=None):
    table, M, tshift = wl.table()
    aE, bE, cE, aB, bB, cB = W.shifted_coeffs(wl.lat, tshift)
    return O.FieldSource(table=table, M=M,
                         coeffs=(aE, bE, cE + bE * shift, aB, bB, cB + bB * shift), atab=atab)


def _gamma_c(st):
    """gamma in the oracle's and the kernels' operation order."""
    return np.sqrt(1.0 + ((st.px * st.px + st.py * st.py) + st.pz * st.pz))


def a_on_lattice(wl, atab, M, coeffs, tau, x):
    """a at time tau dt and position x on the E lattice, linear between
    lattice points (the oracle's own rule for the energy error)."""
    aE, bE, cE = coeffs[0], coeffs[1], coeffs[2]
    m = aE * tau + bE * ((np.asarray(x) - wl.x_origin) / wl.dx - 0.5) + cE
    mf = np.floor(m)
    j0 = mf.astype(np.int64) % M
    j1 = (j0 + 1) % M
    return atab[j0] + (m - mf) * (atab[j1] - atab[j0])


def run_whole(wl, chunk: int = 20000, k_max: int = 12, max_steps: int = 1 << 28,
              energy: bool = False):
    """Returns (state, counters, running max of |R - 1|, largest gamma), and
    with energy=True also the running maximum of the energy error of
    Eq. (gamma error) (a_i: a at the electron's phase when its momentum is
    zero, half a step before the start)."""
    if energy:
        table, M, tshift = wl.table()
        atab, _, _ = wl.potential()
        co = W.shifted_coeffs(wl.lat, tshift)
        fs = O.FieldSource(table=table, M=M, coeffs=co, atab=atab)
        ai = a_on_lattice(wl, atab, M, co, -0.5, wl.x0)
        emax = np.zeros(wl.num)
    else:
        fs = _fields(wl)
        ai = emax = None
    prm = O.make_params(2_000_000, wl.order, wl.dx, wl.dt, wl.psi_max, wl.x_origin, k_max=k_max)
    st = O.State(wl.x0, *wl.p0)
    r0 = O.dephasing_R(st.px, st.py, st.pz)
    rmax = np.zeros(wl.num)
    gmax = _gamma_c(st)
    cnt = O.Counters()
    n = 0
    while n < max_steps:
        O.push(prm, fs, st, n, chunk, counters=cnt, r0=r0, rmax=rmax, gmax=gmax, ai=ai, emax=emax)
        n += chunk
        live = st.status == 0
        if not live.any() or np.all(n * wl.dt - st.x[live] > XI_END):
            break
    if energy:
        return st, cnt, rmax, gmax, emax
    return st, cnt, rmax, gmax


def run_windows(wl, windows, k_max: int = 12, forced_k=None, gamma_max: bool = False,
                energy: bool = False):
    """The oracle over the launches of a device run (n, steps, shift).
    forced_k: optional [total steps, num] int8 array replacing the decision.
    gamma_max: also return the running maximum of gamma (after each step).
    energy: also return the running maximum of the energy error (last)."""
    st = O.State(wl.x0, *wl.p0)
    r0 = O.dephasing_R(st.px, st.py, st.pz)
    rmax = np.zeros(wl.num)
    gmax = _gamma_c(st) if gamma_max else None
    ai = emax = atab = None
    if energy:
        _, M, tshift = wl.table()
        atab, _, _ = wl.potential()
        ai = a_on_lattice(wl, atab, M, W.shifted_coeffs(wl.lat, tshift), -0.5, wl.x0)
        emax = np.zeros(wl.num)
    cnt = O.Counters()
    ktrace = []
    for n, steps, shift in windows:
        prm = O.make_params(wl.ncells, wl.order, wl.dx, wl.dt, wl.psi_max,
                            wl.x_origin + shift * wl.dx, k_max=k_max)
        fk = None if forced_k is None else np.ascontiguousarray(forced_k[n:n + steps])
        kt, pt = O.push(prm, _fields(wl, shift, atab), st, n, steps, counters=cnt, r0=r0,
                        rmax=rmax, gmax=gmax, trace=True, psi_trace=True, forced_k=fk, ai=ai,
                        emax=emax)
        ktrace.append((kt, pt))
    kt = np.concatenate([k for k, _ in ktrace]) if ktrace else np.zeros((0, wl.num), np.int8)
    pt = np.concatenate([p for _, p in ktrace]) if ktrace else np.zeros((0, wl.num))
    return (st, cnt, rmax, kt, pt) + ((gmax,) if gamma_max else ()) + ((emax,) if energy else ())


def moving_windows(wl, S: int = 1000, left: int = 8, k_max: int = 12):
    """The launches a moving-grid run makes (the rule of runner.PulseRun:
    before each launch the grid is shifted so the electron sits `left`
    cells from node 0), found with the oracle itself; returns the windows."""
    st = O.State(wl.x0, *wl.p0)
    windows = []
    n = 0
    while True:
        live = st.status == 0
        if not live.any() or np.all(n * wl.dt - st.x[live] > XI_END):
            break
        shift = int(np.floor((st.x[live].min() - wl.x_origin) / wl.dx)) - left
        prm = O.make_params(wl.ncells, wl.order, wl.dx, wl.dt, wl.psi_max,
                            wl.x_origin + shift * wl.dx, k_max=k_max)
        O.push(prm, _fields(wl, shift), st, n, S)
        windows.append((n, S, shift))
        n += S
    return windows

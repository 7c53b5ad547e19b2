"""Plain FP64 reference of the 1D Yee field solver that feeds the pusher in
the paper's "standard PIC" (Sec. III, Eqs. (Ey) and (Bz)).

TEST INFRASTRUCTURE ONLY: imported by the tests; never by the product path.

Grid and staggering as everywhere in this project: level n holds E_y at
t = n dt on the nodes x = (i + 1/2) dx and B_z at t = (n + 1/2) dt on the
nodes x = i dx, i = 0 .. ncells - 1, in normalised units (c = 1).  With
nu = dt / dx the two updates of Sec. III are

    E^n[i]      = E^{n-1}[i] - nu (B^{n-1/2}[i+1] - B^{n-1/2}[i])
    B^{n+1/2}[i] = B^{n-1/2}[i] - nu (E^n[i] - E^n[i-1])

applied level by level, E first.  The paper does not say how the laser
enters its grid or what happens at the far end; the readings taken here:

* left end (laser injection): B_z at node 0 of every new level is given
  by the caller (a hard source: the incident wave's value there);
* right end: the last E node, which would need B beyond the grid, obeys
  the first-order Mur one-way condition for a wave leaving in +x,
      E^n[N-1] = E^{n-1}[N-2] + kappa (E^n[N-2] - E^{n-1}[N-1]),
      kappa = (dt - dx) / (dt + dx).

Every operation is a plain IEEE double subtract, multiply or add in the
order written above (no fused multiply-add).
"""

from __future__ import annotations

import numpy as np


def coefficients(dx: float, dt: float):
    """(nu, kappa) of the updates above."""
    dx = float(dx)
    dt = float(dt)
    return dt / dx, (dt - dx) / (dt + dx)


def step(E: np.ndarray, B: np.ndarray, nu: float, kappa: float, b0: float):
    """One level: (E^{n-1}, B^{n-1/2}) -> (E^n, B^{n+1/2}); b0 = B^{n+1/2}[0]."""
    E = np.asarray(E, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    En = np.empty_like(E)
    En[:-1] = E[:-1] - nu * (B[1:] - B[:-1])
    En[-1] = E[-2] + kappa * (En[-2] - E[-1])
    Bn = np.empty_like(B)
    Bn[1:] = B[1:] - nu * (En[1:] - En[:-1])
    Bn[0] = b0
    return En, Bn


def advance(E: np.ndarray, B: np.ndarray, dx: float, dt: float, b0_seq):
    """Levels n_first .. n_first + len(b0_seq) - 1 from level n_first - 1
    given as (E, B); b0_seq[c] is B_z at node 0 of level n_first + c.
    Returns (Elev, Blev), arrays [len(b0_seq), ncells]."""
    nu, kappa = coefficients(dx, dt)
    count = len(b0_seq)
    n = len(E)
    if n < 2 or len(B) != n:
        raise ValueError("need two or more nodes and equal E, B lengths")
    Elev = np.empty((count, n))
    Blev = np.empty((count, n))
    e, b = np.asarray(E, dtype=np.float64), np.asarray(B, dtype=np.float64)
    for c in range(count):
        e, b = step(e, b, nu, kappa, float(b0_seq[c]))
        Elev[c] = e
        Blev[c] = b
    return Elev, Blev


def advance_lattice(E: np.ndarray, B: np.ndarray, dx: float, dt: float, n_first: int,
                    count: int, table: np.ndarray, aB: int, cB: int):
    """advance() with the source taken from a phase table, as the library's
    call takes it: B_z at node 0 of level m is table[(aB m + cB) mod M]."""
    M = len(table)
    b0 = [table[(aB * m + cB) % M] for m in range(n_first, n_first + count)]
    return advance(E, B, dx, dt, b0)

"""Seeded synthetic inputs: particle loads and plane-wave field lattices.

This module is the only code shared by the product path and the FP64
oracle.  It draws random numbers and tabulates the prescribed laser field;
it holds none of the integrator's arithmetic (no interpolation, no
gather, no push, no sub-cycling decision).

Units are normalised: t in 1/omega, x in c/omega, p in m c, fields in
m omega c / |e|.  The wavelength and the period are both 2 pi.

Field model (Sec. II, Eqs. (laser5)-(laser3)): E_y = B_z = -da/dxi with
xi = t - x.  ``kind='flat'`` uses a = a0 sin(xi); ``kind='gauss'`` uses the
paper's envelope a = a0 exp(-(xi - xi0)^2 / (2 sigma^2)) sin(xi).

Yee lattice.  With dx = (R/Q) dt for integers R and Q, every E_y sample
(x = x_origin + (i + 1/2) dx, t = n dt) and every B_z sample
(x = x_origin + i dx, t = (n + 1/2) dt) sits on the phase lattice
xi_m = m * dt / (2 Q), so a level can be filled from one table by an affine
index m = a n + b i + c.  For the paper's c dt / dx = 1/1.01 (Sec. IV:
lambda/dx = 74.26 at T/dt = 75), R/Q = 101/100.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass(frozen=True)
class Lattice:
    """Affine map from (level n, node i) to a phase-table index."""

    q: int            # dt = 2 q lattice units
    r: int            # dx = 2 r lattice units
    j0: int           # x_origin = -j0 lattice units (phase reference at x=0)
    n_t: int          # steps per laser period, dt = 2 pi / n_t
    # E_y(n, i) = table[(aE n + bE i + cE) mod M], same for B_z
    aE: int
    bE: int
    cE: int
    aB: int
    bB: int
    cB: int

    @property
    def dt(self) -> float:
        return TWO_PI / self.n_t

    @property
    def dx(self) -> float:
        return self.dt * self.r / self.q

    @property
    def unit(self) -> float:
        """Phase step of one lattice unit."""
        return self.dt / (2 * self.q)

    @property
    def x_origin(self) -> float:
        return -self.j0 * self.unit

    @property
    def period(self) -> int:
        """Lattice units per laser period (table length of a flat wave)."""
        return 2 * self.q * self.n_t

    def coeffs(self):
        return (self.aE, self.bE, self.cE, self.aB, self.bB, self.cB)


def yee_lattice(n_t: int, r: int = 101, q: int = 100, j0: int = 0) -> Lattice:
    """Lattice for dt = 2 pi / n_t and dx = (r / q) dt.

    xi_E(n, i) = n dt - x_origin - (i + 1/2) dx  -> m = 2 q n - 2 r i - r + j0
    xi_B(n, i) = (n + 1/2) dt - x_origin - i dx -> m = 2 q n + q - 2 r i + j0
    """
    return Lattice(q=q, r=r, j0=j0, n_t=n_t,
                   aE=2 * q, bE=-2 * r, cE=-r + j0,
                   aB=2 * q, bB=-2 * r, cB=q + j0)


GAUSS_XI0 = 160.0 * math.pi      # pulse centre, relative to the electrons' initial phase
GAUSS_SIGMA = 8.0 * math.pi
GAUSS_MARGIN = 64.0 * math.pi    # phase covered beyond the pulse on either side


def plane_wave_table(lat: Lattice, a0: float, kind: str = "flat",
                     xi0: float = GAUSS_XI0, sigma: float = GAUSS_SIGMA,
                     m_lo: int | None = None, m_count: int | None = None):
    """Table of E_y = B_z = -da/dxi on the lattice.

    Returns (table, M, shift): the value at lattice index m is
    table[(m - shift) mod M].  For a flat wave M is one period and
    shift = 0.  For the Gaussian pulse the table spans m_count points
    starting at m_lo (by default the phases -GAUSS_MARGIN .. xi0 + 9 sigma +
    GAUSS_MARGIN, so that no node of a grid near the electrons wraps
    around), and shift = m_lo.
    """
    if kind == "flat":
        m = np.arange(lat.period, dtype=np.int64)
        xi = m.astype(np.float64) * lat.unit
        return -a0 * np.cos(xi), lat.period, 0
    if kind == "gauss":
        if m_lo is None:
            m_lo = -int(math.ceil(GAUSS_MARGIN / lat.unit))
        if m_count is None:
            m_count = int(math.ceil((xi0 + 9.0 * sigma + GAUSS_MARGIN) / lat.unit)) - m_lo + 1
        m = np.arange(m_lo, m_lo + m_count, dtype=np.int64)
        xi = m.astype(np.float64) * lat.unit
        env = np.exp(-((xi - xi0) ** 2) / (2.0 * sigma * sigma))
        # -da/dxi for a = a0 env sin(xi)
        dadxi = a0 * env * (np.cos(xi) - (xi - xi0) / (sigma * sigma) * np.sin(xi))
        return -dadxi, m_count, m_lo
    raise ValueError(f"unknown wave kind {kind!r}")


def potential_table(lat: Lattice, a0: float, kind: str = "flat",
                    xi0: float = GAUSS_XI0, sigma: float = GAUSS_SIGMA,
                    m_lo: int | None = None, m_count: int | None = None):
    """The vector potential a itself on the lattice of plane_wave_table, with
    the same (table, M, shift) layout (for the energy error of the model
    problem, whose analytic gamma is 1 + (a - a_i)^2 / 2)."""
    if kind == "flat":
        m = np.arange(lat.period, dtype=np.int64)
        xi = m.astype(np.float64) * lat.unit
        return a0 * np.sin(xi), lat.period, 0
    if kind == "gauss":
        if m_lo is None:
            m_lo = -int(math.ceil(GAUSS_MARGIN / lat.unit))
        if m_count is None:
            m_count = int(math.ceil((xi0 + 9.0 * sigma + GAUSS_MARGIN) / lat.unit)) - m_lo + 1
        m = np.arange(m_lo, m_lo + m_count, dtype=np.int64)
        xi = m.astype(np.float64) * lat.unit
        return a0 * np.exp(-((xi - xi0) ** 2) / (2.0 * sigma * sigma)) * np.sin(xi), m_count, m_lo
    raise ValueError(f"unknown wave kind {kind!r}")


def shifted_coeffs(lat: Lattice, shift: int):
    """Lattice coefficients with a table shift folded into c."""
    aE, bE, cE, aB, bB, cB = lat.coeffs()
    return (aE, bE, cE - shift, aB, bB, cB - shift)


def sample_levels(lat: Lattice, table: np.ndarray, M: int, shift: int,
                  ncells: int, n_first: int, count: int):
    """Explicit E_y and B_z arrays [count, ncells] for levels n_first..

    Pure table indexing (the same values the device-side lattice sampler
    writes).  Used to hand identical fields to the oracle and the GPU.
    """
    aE, bE, cE, aB, bB, cB = shifted_coeffs(lat, shift)
    n = np.arange(n_first, n_first + count, dtype=np.int64)[:, None]
    i = np.arange(ncells, dtype=np.int64)[None, :]
    E = table[np.mod(aE * n + bE * i + cE, M)]
    B = table[np.mod(aB * n + bB * i + cB, M)]
    return np.ascontiguousarray(E), np.ascontiguousarray(B)


def uniform_positions(num: int, x_lo: float, span: float, seed: int) -> np.ndarray:
    """x0 ~ U[x_lo, x_lo + span), drawn with PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return x_lo + span * rng.random(num)


def thermal_momenta(num: int, theta: float, seed: int) -> np.ndarray:
    """Non-relativistic Maxwellian: each component ~ N(0, sqrt(theta)).

    theta = k T / (m c^2) (10 keV -> 10 / 511).  Returns [3, num].
    """
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    return math.sqrt(theta) * rng.standard_normal((3, num))


@dataclasses.dataclass
class Workload:
    """One particle load in a prescribed plane wave."""

    name: str
    num: int
    a0: float
    n_t: int
    ncells: int
    steps: int
    order: int
    psi_max: float
    x0: np.ndarray
    p0: np.ndarray            # [3, num]
    lat: Lattice
    kind: str = "flat"

    @property
    def dt(self) -> float:
        return self.lat.dt

    @property
    def dx(self) -> float:
        return self.lat.dx

    @property
    def x_origin(self) -> float:
        return self.lat.x_origin

    def table(self):
        return plane_wave_table(self.lat, self.a0, self.kind)

    def potential(self):
        return potential_table(self.lat, self.a0, self.kind)


def make_workload(name: str, num: int, a0: float, n_t: int, ncells: int,
                  periods: float, order: int, psi_max: float, span_lambda: float,
                  seed: int, theta: float = 0.0, margin_cells: int = 4) -> Workload:
    """Electrons spread uniformly over ``span_lambda`` wavelengths starting
    ``margin_cells`` cells from the left edge, at rest unless theta > 0."""
    lat = yee_lattice(n_t)
    x_lo = lat.x_origin + margin_cells * lat.dx
    x0 = uniform_positions(num, x_lo, span_lambda * TWO_PI, seed)
    if theta > 0.0:
        p0 = thermal_momenta(num, theta, seed)
    else:
        p0 = np.zeros((3, num))
    steps = int(round(periods * n_t))
    return Workload(name=name, num=num, a0=a0, n_t=n_t, ncells=ncells, steps=steps,
                    order=order, psi_max=psi_max, x0=x0, p0=p0, lat=lat)


# Workloads with the shapes of the paper's model problem (a test electron
# population in a linearly polarised plane wave, Sec. II) at production sizes.
def small_case(order: int = 3, num: int = 1024, periods: float = 20.0) -> Workload:
    """1024 electrons at rest over one wavelength, a0 = 10, T/dt = 75,
    2048 cells, 20 periods, psi_max = 0.01."""
    return make_workload("a0=10 P=1024 T/dt=75 cells=2048", num, 10.0, 75, 2048,
                         periods, order, 0.01, 1.0, seed=1)


LARGE_A0 = {20: 30.0, 21: 100.0, 22: 150.0}


def large_case(seed: int = 22, num: int = 1 << 20, periods: float = 100.0,
               order: int = 3) -> Workload:
    """2^20 electrons at rest over 8 wavelengths, a0 in {30, 100, 150} by seed,
    T/dt = 75, 8192 cells, 100 periods, 3rd order, psi_max = 0.01."""
    a0 = LARGE_A0[seed]
    return make_workload(f"a0={a0:g} P={num} T/dt=75 cells=8192", num, a0, 75, 8192,
                         periods, order, 0.01, 8.0, seed=seed)


def predictor_case(num: int = 1 << 22, periods: float = 100.0, order: int = 3) -> Workload:
    """The learned-binning workload: 2^22 electrons at rest over 16
    wavelengths in an a0 = 150 plane wave, T/dt = 75, 16384 cells, 100
    periods, 3rd order, psi_max = 0.01."""
    return make_workload(f"predictor a0=150 P={num} cells=16384", num, 150.0, 75, 16384,
                         periods, order, 0.01, 16.0, seed=9)


def stress_case(psi_max: float = 0.01, num: int = 1 << 24, periods: float = 100.0,
                order: int = 3) -> Workload:
    """2^24 thermal electrons (10 keV) over 200 wavelengths, a0 = 150,
    65536 cells, 3rd order by default."""
    return make_workload(f"stress psi={psi_max:g} P={num}", num, 150.0, 75, 65536,
                         periods, order, psi_max, 200.0, seed=5, theta=10.0 / 511.0)


def pulse_case(a0: float, n_t: int = 75, order: int = 3, psi_max: float = 0.01, num: int = 1,
               ncells: int = 1100) -> Workload:
    """The paper's model problem (Sec. II): electrons at rest at x = 0, t = 0
    hit by the Gaussian pulse a = a0 exp(-(xi - xi0)^2 / (2 sigma^2)) sin(xi),
    xi = t - x, xi0 = 160 pi after the electrons' initial phase, sigma = 8 pi.
    dt = 2 pi / n_t, dx = 1.01 dt.  The grid of ncells nodes starts eight
    cells to the left of the electrons and is moved along with them; the run
    lasts until the pulse has passed (steps = 0: decided by the driver)."""
    lat = yee_lattice(n_t, j0=8 * 2 * 101)        # x_origin = -8 dx
    return Workload(name=f"pulse a0={a0:g} T/dt={n_t} order {order} psi={psi_max:g}",
                    num=num, a0=a0, n_t=n_t, ncells=ncells, steps=0, order=order,
                    psi_max=psi_max, x0=np.zeros(num), p0=np.zeros((3, num)), lat=lat,
                    kind="gauss")


def batch_case(seed: int = 3, nruns: int = 64, periods: float = 50.0,
               p_range=(1e3, 4e6), a0_range=(1.0, 150.0), n_t_choices=(40, 75, 150),
               cells_range=(2048, 16384), span_lambda: float = 1.0, scale: float = 1.0):
    """Independent runs of uneven size: particle counts log-uniform in p_range
    (times `scale`), a0 log-uniform in a0_range, T/dt drawn from
    n_t_choices, grids log-uniform in cells_range and enlarged where the run
    needs more room (x0 span + periods wavelengths + margins), electrons at
    rest over `span_lambda` wavelengths, 3rd order, psi_max = 0.01."""
    rng = np.random.Generator(np.random.PCG64(seed))
    runs = []
    for r in range(nruns):
        num = max(1, int(round(scale * math.exp(rng.uniform(math.log(p_range[0]),
                                                            math.log(p_range[1]))))))
        a0 = math.exp(rng.uniform(math.log(a0_range[0]), math.log(a0_range[1])))
        n_t = int(n_t_choices[int(rng.integers(0, len(n_t_choices)))])
        cells = int(round(math.exp(rng.uniform(math.log(cells_range[0]),
                                               math.log(cells_range[1])))))
        need = int(math.ceil((span_lambda + periods + 0.5) * n_t * 100 / 101)) + 16
        cells = max(cells, need)
        wl = make_workload(f"run{r} a0={a0:.3g} T/dt={n_t}", num, a0, n_t, cells, periods,
                           3, 0.01, span_lambda, seed=1000 * seed + r)
        runs.append(wl)
    return runs

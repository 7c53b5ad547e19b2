"""Drive a workload through the C ABI: field lattice on the device, ring
preload, chunks of S steps.  Argument marshalling and loop control only."""

from __future__ import annotations

import numpy as np

from . import picsub
from . import workloads as W


class DeviceRun:
    """A Pusher bound to one workload, with its phase table on the device.

    fields="lattice": every level sampled from the phase table (the
    prescribed wave, "perfectly propagating PIC").  fields="yee": levels
    -order .. 0 sampled, every later level made by the Yee solver with the
    wave entering at node 0 ("standard PIC")."""

    def __init__(self, wl: W.Workload, *, S: int = 1, order: int | None = None,
                 psi_max: float | None = None, precision: str = "fp64", binning: str = "ballot",
                 k_max: int = 8, ring_extra: int = 0, stream=None, fields: str = "lattice"):
        import torch
        if fields not in ("lattice", "yee"):
            raise ValueError("fields must be 'lattice' or 'yee'")
        self.torch = torch
        self.fields = fields
        self.wl = wl
        self.order = wl.order if order is None else order
        self.S = int(S)
        self.psi_max = wl.psi_max if psi_max is None else psi_max
        table, M, shift = wl.table()
        self.M = int(M)
        self.coeffs = W.shifted_coeffs(wl.lat, shift)
        self.table = torch.from_numpy(np.ascontiguousarray(table)).to("cuda")
        self.pusher = picsub.Pusher(num=wl.num, ncells=wl.ncells, order=self.order, dx=wl.dx,
                                    dt=wl.dt, psi_max=self.psi_max, x_origin=wl.x_origin,
                                    k_max=k_max, ring_depth=self.S + self.order + ring_extra,
                                    precision=precision, binning=binning, stream=stream)
        dev = "cuda"
        self.x0 = torch.from_numpy(np.ascontiguousarray(wl.x0)).to(dev)
        self.p0 = [torch.from_numpy(np.ascontiguousarray(wl.p0[c])).to(dev) for c in range(3)]
        self.k0 = None

    def reset(self, k_old=None):
        """Load the initial state (device to device) and the first levels."""
        self.pusher.particles_set(self.x0, *self.p0, k_old)
        # levels -hist .. -1 (the push needs -order; the predictor's features
        # read -2 as well), and level 0 when the Yee solver makes the rest
        extra = 1 if self.fields == "yee" else 0
        hist = max(self.order, 2)
        if hist + extra > self.pusher.ring_depth:
            hist = self.order
        self.pusher.fields_load_lattice(-hist, hist + extra, self.table, self.M, self.coeffs)
        self.n = 0

    def advance(self, steps: int, S: int | None = None):
        """Advance `steps` steps of size dt in chunks of S (asynchronous)."""
        S = self.S if S is None else S
        end = self.n + steps
        while self.n < end:
            s = min(S, end - self.n)
            self.fill(self.n, s)
            self.pusher.push(self.n, s)
            self.n += s

    def fill(self, n: int, s: int):
        """Put levels n .. n + s - 1 into the ring."""
        if self.fields == "lattice":
            self.pusher.fields_load_lattice(n, s, self.table, self.M, self.coeffs)
        else:
            lo = max(n, 1)              # level 0 was sampled by reset()
            if n + s > lo:
                self.pusher.fields_yee(lo, n + s - lo, self.table, self.M, self.coeffs[3],
                                       self.coeffs[5])

    def diag(self):
        return self.pusher.diag()

    def close(self):
        self.pusher.close()


class BatchRun:
    """Many workloads in one context, advanced by device-driven windows of S
    steps (each run stops at its own step count); optionally captured into a
    HIP graph that replays a whole pass."""

    def __init__(self, wls, *, S: int = 250, precision: str = "fp64fast",
                 binning: str = "none", k_max: int = 8, stream=None):
        import torch
        self.torch = torch
        self.wls = list(wls)
        self.S = int(S)
        order = self.wls[0].order
        runs = []
        self.tables = []
        for wl in self.wls:
            assert wl.order == order
            runs.append((wl.num, picsub.make_params(
                ncells=wl.ncells, order=order, dx=wl.dx, dt=wl.dt, psi_max=wl.psi_max,
                x_origin=wl.x_origin, k_max=k_max, ring_depth=self.S + order,
                precision=precision, binning=binning)))
            table, M, shift = wl.table()
            self.tables.append((torch.from_numpy(np.ascontiguousarray(table)).to("cuda"), int(M),
                                W.shifted_coeffs(wl.lat, shift)))
        self.pusher = picsub.Pusher(runs=runs, stream=stream)
        self.x0 = torch.from_numpy(np.concatenate([wl.x0 for wl in self.wls])).to("cuda")
        self.p0 = [torch.from_numpy(np.concatenate([wl.p0[c] for wl in self.wls])).to("cuda")
                   for c in range(3)]
        self.max_steps = max(wl.steps for wl in self.wls)
        self.windows = (self.max_steps + self.S - 1) // self.S

    @property
    def sub_steps_hint(self):
        return None

    def reset(self):
        self.pusher.particles_set(self.x0, *self.p0)
        for r, (wl, (tab, M, co)) in enumerate(zip(self.wls, self.tables)):
            self.pusher.source_set(r, 0, tab, M, co, n_stop=wl.steps)

    def run_all(self):
        """One full pass: every run to its own last step (asynchronous)."""
        for _ in range(self.windows):
            self.pusher.advance(self.S)

    def capture(self):
        self.pusher.graph_capture(self.S, self.windows)

    def replay(self):
        self.pusher.graph_launch()

    def diag(self):
        return self.pusher.diag()

    def close(self):
        self.pusher.close()


def initial_potential(wl: W.Workload, atab, M: int, coeffs):
    """a_i of every electron of a pulse workload: the potential at its start
    position half a step before the start (the time of its zero momentum),
    linear between the points of the potential lattice (A, B, C) = coeffs[:3]."""
    A, B, Cc = coeffs[:3]
    m = A * -0.5 + B * ((wl.x0 - wl.x_origin) / wl.dx - 0.5) + Cc
    mf = np.floor(m)
    j0 = mf.astype(np.int64) % M
    j1 = (j0 + 1) % M
    return atab[j0] + (m - mf) * (atab[j1] - atab[j0])


def pulse_passed(wl: W.Workload, n: int, x, status) -> bool:
    """True once no electron is live or the pulse (phase t - x) has passed
    every live one: the end of a model-problem run."""
    live = status == 0
    if not live.any():
        return True
    return bool(np.all(n * wl.dt - x[live] > W.GAUSS_XI0 + 7.0 * W.GAUSS_SIGMA))


class PulseRun:
    """Electrons in the Gaussian pulse of the paper's model problem (Sec. II),
    pushed in launches of S steps on a grid of wl.ncells nodes that moves with
    them: before each launch the grid is shifted (pic_grid_shift) so that the
    leftmost live electron sits `left` cells from node 0, and the levels of
    the launch are sampled for the moved nodes.  The run ends once the pulse
    has passed every live electron (phase t - x beyond xi0 + 7 sigma).

    Records, for the caller: the shift and length of every launch (so that a
    reference can repeat the same grids) and, through the trajectory
    diagnostics, the running maxima of |R - 1| (the dephasing error of
    Sec. IV, Eq. (R error)), of gamma (the peak energy of Sec. IV) and, with
    energy=True, of the energy error of Eq. (gamma error) against the
    plane-wave solution (the potential table of the same lattice, a_i at each
    electron's phase half a step before the start)."""

    def __init__(self, wl: W.Workload, *, S: int = 1000, precision: str = "fp64fast",
                 k_max: int = 12, left: int = 8, stream=None, energy: bool = False):
        import torch
        if wl.kind != "gauss":
            raise ValueError("PulseRun drives the Gaussian pulse workload")
        if wl.ncells < left + int(S * wl.dt / wl.dx) + 16:
            raise ValueError("the grid is too short for S steps")
        self.torch = torch
        self.wl = wl
        self.S = int(S)
        self.left = int(left)
        table, M, shift = wl.table()
        self.M = int(M)
        self.coeffs = W.shifted_coeffs(wl.lat, shift)
        self.table = torch.from_numpy(np.ascontiguousarray(table)).to("cuda")
        self.energy = bool(energy)
        if self.energy:
            atab, aM, ashift = wl.potential()
            if aM != self.M or ashift != shift:
                raise ValueError("the potential table must share the field table's lattice")
            self.atab = torch.from_numpy(np.ascontiguousarray(atab)).to("cuda")
            self.ai = initial_potential(wl, atab, aM, self.coeffs)
        self.pusher = picsub.Pusher(num=wl.num, ncells=wl.ncells, order=wl.order, dx=wl.dx,
                                    dt=wl.dt, psi_max=wl.psi_max, x_origin=wl.x_origin,
                                    k_max=k_max, ring_depth=self.S + wl.order,
                                    precision=precision, binning="none", stream=stream)
        self.shift = 0
        self.n = 0
        self.windows = []            # (n, steps, shift) of every launch

    def reset(self):
        if self.shift:
            self.pusher.grid_shift(-self.shift)
            self.shift = 0
        self.pusher.particles_set(self.wl.x0, *self.wl.p0)
        self.pusher.diag_track(True)
        if self.energy:
            self.pusher.gamma_error_start(self.ai)
        self.n = 0
        self.windows = []

    def window(self) -> bool:
        """One launch; False once the pulse has passed every live electron."""
        wl = self.wl
        d = self.pusher.diag()
        if pulse_passed(wl, self.n, d["x"], d["status"]):
            return False
        live = d["status"] == 0
        target = int(np.floor((d["x"][live].min() - wl.x_origin) / wl.dx)) - self.left
        if target != self.shift:
            self.pusher.grid_shift(target - self.shift)
            self.shift = target
        aE, bE, cE, aB, bB, cB = self.coeffs
        co = (aE, bE, cE + bE * self.shift, aB, bB, cB + bB * self.shift)
        p = wl.order
        self.pusher.fields_load_lattice(self.n - p, p + self.S, self.table, self.M, co)
        if self.energy:
            self.pusher.gamma_error_lattice(self.atab, self.M, co[:3])
        self.pusher.push(self.n, self.S)
        self.windows.append((self.n, self.S, self.shift))
        self.n += self.S
        return True

    def run(self, max_steps: int = 1 << 31):
        while self.n < max_steps and self.window():
            pass
        return self

    def results(self) -> dict:
        d = self.pusher.diag()
        r0, rmax = self.pusher.dephasing_read()
        out = {"diag": d, "eps_dephasing": rmax, "R0": r0,
               "gamma_max": self.pusher.gamma_max_read(),
               "steps": self.n, "windows": list(self.windows)}
        if self.energy:
            out["eps_energy"] = self.pusher.gamma_error_read()
        return out

    def close(self):
        self.pusher.close()


class PulseBatch:
    """Several runs of the model problem (one pulse workload per run, all of
    one interpolation order) in one batch context, pushed together in
    launches of S steps.  Before each launch every run's grid is moved so
    that its leftmost live electron sits `left` cells from node 0 (the rule of
    PulseRun) and the run's levels are sampled for the moved nodes.  A run is
    finished at the first launch boundary where the pulse has passed its
    electrons, or where it has taken step_cap[r] steps (an electron that the
    integrator's errors keep riding with the pulse): its results are read
    then ("pulse_passed" tells which), and it is pushed on with the others
    (nothing it recorded changes).  The batch ends when every run is
    finished.  With energy=True the energy error of Eq. (gamma error) is
    kept as well."""

    def __init__(self, wls, *, S: int = 1000, precision: str = "fp64", k_max: int = 12,
                 left: int = 8, energy: bool = True, step_cap=None, stream=None):
        import torch
        self.wls = list(wls)
        order = self.wls[0].order
        for wl in self.wls:
            if wl.kind != "gauss" or wl.order != order:
                raise ValueError("a pulse batch holds Gaussian-pulse workloads of one order")
            if wl.ncells < left + int(S * wl.dt / wl.dx) + 16:
                raise ValueError("a grid is too short for S steps")
        self.S, self.left, self.order, self.energy = int(S), int(left), order, bool(energy)
        self.src = []           # (table, M, coeffs, potential table) per run
        ai = []
        runs = []
        for wl in self.wls:
            table, M, shift = wl.table()
            co = W.shifted_coeffs(wl.lat, shift)
            atab = None
            if self.energy:
                at, aM, ashift = wl.potential()
                if aM != M or ashift != shift:
                    raise ValueError("the potential table must share the field table's lattice")
                atab = torch.from_numpy(np.ascontiguousarray(at)).to("cuda")
                ai.append(initial_potential(wl, at, M, co))
            self.src.append((torch.from_numpy(np.ascontiguousarray(table)).to("cuda"), int(M),
                             co, atab))
            runs.append((wl.num, picsub.make_params(
                ncells=wl.ncells, order=order, dx=wl.dx, dt=wl.dt, psi_max=wl.psi_max,
                x_origin=wl.x_origin, k_max=k_max, ring_depth=self.S + order,
                precision=precision, binning="none")))
        self.pusher = picsub.Pusher(runs=runs, stream=stream)
        self.first = np.cumsum([0] + [wl.num for wl in self.wls])
        self.ai = np.concatenate(ai) if self.energy else None
        self.shift = [0] * len(self.wls)
        self.step_cap = [None] * len(self.wls) if step_cap is None else list(step_cap)

    def reset(self):
        for r, sh in enumerate(self.shift):
            if sh:
                self.pusher.grid_shift(-sh, run=r)
        self.shift = [0] * len(self.wls)
        self.pusher.particles_set(np.concatenate([wl.x0 for wl in self.wls]),
                                  *[np.concatenate([wl.p0[c] for wl in self.wls])
                                    for c in range(3)])
        self.pusher.diag_track(True)
        if self.energy:
            self.pusher.gamma_error_start(self.ai)
        self.n = 0
        self.windows = [[] for _ in self.wls]     # (n, steps, shift) of each run's launches
        self.results = [None] * len(self.wls)

    def _record(self, r, d, passed):
        sl = slice(int(self.first[r]), int(self.first[r + 1]))
        _, rmax = self.pusher.dephasing_read()
        out = {"steps_run": self.n, "pulse_passed": passed, "windows": list(self.windows[r]),
               "counters": self.pusher.run_counters(r),
               "x": d["x"][sl], "px": d["px"][sl], "py": d["py"][sl], "pz": d["pz"][sl],
               "status": d["status"][sl], "eps_dephasing": rmax[sl],
               "gamma_max": self.pusher.gamma_max_read()[sl]}
        if self.energy:
            out["eps_energy"] = self.pusher.gamma_error_read()[sl]
        return out

    def window(self) -> bool:
        """One launch of every run; False once every run is finished."""
        d = self.pusher.diag()
        for r, wl in enumerate(self.wls):
            sl = slice(int(self.first[r]), int(self.first[r + 1]))
            if self.results[r] is not None:
                continue
            passed = pulse_passed(wl, self.n, d["x"][sl], d["status"][sl])
            cap = self.step_cap[r]
            if passed or (cap is not None and self.n >= cap):
                self.results[r] = self._record(r, d, passed)
        if all(res is not None for res in self.results):
            return False
        p = self.order
        for r, wl in enumerate(self.wls):
            sl = slice(int(self.first[r]), int(self.first[r + 1]))
            live = d["status"][sl] == 0
            if live.any():
                target = int(np.floor((d["x"][sl][live].min() - wl.x_origin) / wl.dx)) - self.left
                if target != self.shift[r]:
                    self.pusher.grid_shift(target - self.shift[r], run=r)
                    self.shift[r] = target
            table, M, co, atab = self.src[r]
            sh = self.shift[r]
            cos = (co[0], co[1], co[2] + co[1] * sh, co[3], co[4], co[5] + co[4] * sh)
            self.pusher.fields_load_lattice_r(r, self.n - p, p + self.S, table, M, cos)
            if self.energy:
                self.pusher.gamma_error_lattice(atab, M, cos[:3], run=r)
            if self.results[r] is None:
                self.windows[r].append((self.n, self.S, sh))
        self.pusher.push(self.n, self.S)
        self.n += self.S
        return True

    def unfinished(self) -> int:
        return sum(res is None for res in self.results)

    def run(self, max_steps: int = 1 << 40):
        while self.n < max_steps and self.window():
            pass
        return self.results

    def close(self):
        self.pusher.close()


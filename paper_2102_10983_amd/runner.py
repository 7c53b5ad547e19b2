"""Drive a workload through the C ABI: field lattice on the device, ring
preload, chunks of S steps.  Argument marshalling and loop control only."""

from __future__ import annotations

import numpy as np

from . import picsub
from . import workloads as W


class DeviceRun:
    """A Pusher bound to one workload, with its phase table on the device."""

    def __init__(self, wl: W.Workload, *, S: int = 1, order: int | None = None,
                 psi_max: float | None = None, precision: str = "fp64", binning: str = "ballot",
                 k_max: int = 8, ring_extra: int = 0, stream=None):
        import torch
        self.torch = torch
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
        self.pusher.fields_load_lattice(-self.order, self.order, self.table, self.M, self.coeffs)
        self.n = 0

    def advance(self, steps: int, S: int | None = None):
        """Advance `steps` steps of size dt in chunks of S (asynchronous)."""
        S = self.S if S is None else S
        end = self.n + steps
        while self.n < end:
            s = min(S, end - self.n)
            self.pusher.fields_load_lattice(self.n, s, self.table, self.M, self.coeffs)
            self.pusher.push(self.n, s)
            self.n += s

    def diag(self):
        return self.pusher.diag()

    def close(self):
        self.pusher.close()

"""The accuracy and cost study of the model problem from GPU runs: one
electron at rest hit by the Gaussian pulse of Sec. II, over a0, the
interpolation order (Sec. IV-VII), sub-cycling on or off (Psi_max = 0.01 or
none) and the resolution T/dt.  Each (order, T/dt) pair is one batch context
(runner.PulseBatch) holding every a0 with and without sub-cycling.

Reported per run: epsilon_dephasing (Eq. (R error)), epsilon_energy
(Eq. (gamma error)), the peak gamma, N and N* (Sec. VII) and
delta_steps = N* / (N* + N); derived: chi^3 = eps^1 / eps^3 and
chi^5 = eps^1 / eps^5 with sub-cycling (Sec. VII).

    python -m paper_2102_10983_amd.pulse_sweep [--a0 5 10 25 50 75 100]
        [--orders 1 2 3 5] [--nt 75 150 600] [--precision fp64|fp64fast]
        [--json out.json]
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

from . import runner
from . import workloads as W

SUB_PSI = 0.01         # Psi_max with sub-cycling (Sec. V)
NO_SUB = 1e30          # no sub-cycling: k = 0 at every step


def window_steps(n_t: int) -> tuple[int, int]:
    """(steps per launch, grid nodes) for resolution T/dt = n_t: about ten
    wavelengths of travel per launch, on a grid long enough for it."""
    S = 10 * n_t
    cells = int(math.ceil(S * 100 / 101)) + 40
    return S, cells


def analytic_steps(a0: float, n_t: int) -> int:
    """Steps until the pulse has passed an electron that follows the
    plane-wave solution: phase xi_end = xi0 + 7 sigma reached at time
    t = xi_end + x, x = (1/2) int (a - a_i)^2 dxi = a0^2 sigma sqrt(pi) / 4
    (App. A, with a_i = 0 for an electron the pulse has not reached)."""
    t = W.GAUSS_XI0 + 7.0 * W.GAUSS_SIGMA + a0 * a0 * W.GAUSS_SIGMA * math.sqrt(math.pi) / 4
    return int(math.ceil(t / (2.0 * math.pi / n_t)))


def run_batch(a0s, order: int, n_t: int, precision: str = "fp64", subs=(True, False),
              say=None, cap_factor: float = 3.0):
    """Every a0, with and without sub-cycling, at one order and resolution;
    a list of records.  A run is stopped after cap_factor times the steps of
    the plane-wave solution (record "pulse_passed" False: an electron that
    the integrator's errors keep riding with the pulse)."""
    S, cells = window_steps(n_t)
    cases = [(a0, sub) for sub in subs for a0 in a0s]
    wls = [W.pulse_case(a0, n_t, order, SUB_PSI if sub else NO_SUB, ncells=cells)
           for a0, sub in cases]
    caps = [int(cap_factor * analytic_steps(a0, n_t)) for a0, _ in cases]
    b = runner.PulseBatch(wls, S=S, precision=precision, energy=True, step_cap=caps)
    t0 = last = time.perf_counter()
    try:
        b.reset()
        while b.window():
            if say and time.perf_counter() - last > 20.0:
                last = time.perf_counter()
                say(f"  order {order}, T/dt {n_t}: step {b.n}, {b.unfinished()} runs left")
        res = b.results
    finally:
        b.close()
    out = []
    for (a0, sub), r in zip(cases, res):
        c = r["counters"]
        n, ns = c["steps"], c["n_star"]
        out.append({"a0": a0, "order": order, "n_t": n_t, "subcycling": sub,
                    "pulse_passed": bool(r["pulse_passed"]),
                    "psi_max": SUB_PSI if sub else None, "precision": precision,
                    "eps_dephasing": float(r["eps_dephasing"][0]),
                    "eps_energy": float(r["eps_energy"][0]),
                    "gamma_max_over_analytic": float(r["gamma_max"][0]) / (1.0 + a0 * a0 / 2),
                    "steps": int(n), "n_star": int(ns), "sub_steps": int(c["sub_steps"]),
                    "delta_steps": ns / (ns + n) if n else 0.0,
                    "lost": int(c["lost"]), "launches": len(r["windows"])})
    if say:
        say(f"order {order}, T/dt {n_t}: {len(cases)} runs in {time.perf_counter() - t0:.1f} s")
    return out


def chi(records, p: int) -> dict:
    """chi^p = eps^1 / eps^p (with sub-cycling) per (T/dt, a0)."""
    eps = {(r["order"], r["n_t"], r["a0"]): r["eps_dephasing"]
           for r in records if r["subcycling"]}
    out = {}
    for (o, n_t, a0), e in eps.items():
        if o == p and (1, n_t, a0) in eps and e > 0:
            out[(n_t, a0)] = eps[(1, n_t, a0)] / e
    return out


def sweep(a0s=(5.0, 10.0, 25.0, 50.0, 75.0, 100.0), orders=(1, 2, 3, 5),
          n_ts=(75, 150, 600), precision: str = "fp64", say=None):
    recs = []
    for n_t in n_ts:
        for order in orders:
            recs += run_batch(a0s, order, n_t, precision, say=say)
    return recs


def _table(recs, say):
    say("order  T/dt  sub   a0    eps_deph   eps_energy  gmax/th   N          N*         delta")
    for r in recs:
        say(f"{r['order']:5d} {r['n_t']:5d} {'on ' if r['subcycling'] else 'off'} {r['a0']:5g} "
            f"{r['eps_dephasing']:10.4g} {r['eps_energy']:11.4g} {r['gamma_max_over_analytic']:8.3f} "
            f"{r['steps']:10d} {r['n_star']:10d} {r['delta_steps']:7.4f}"
            + ("" if r["pulse_passed"] else "  (pulse never passed: stopped)"))
    for p in (3, 5):
        c = chi(recs, p)
        if c:
            say(f"chi^{p}: " + ", ".join(f"T/dt {n_t} a0 {a0:g}: {v:.3g}"
                                         for (n_t, a0), v in sorted(c.items())))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--a0", type=float, nargs="+", default=[5, 10, 25, 50, 75, 100])
    ap.add_argument("--orders", type=int, nargs="+", default=[1, 2, 3, 5])
    ap.add_argument("--nt", type=int, nargs="+", default=[75, 150, 600])
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp64fast"))
    ap.add_argument("--json", default=None, help="write the records to this file")
    args = ap.parse_args(argv)

    def say(*a):
        print(*a, flush=True)
    recs = sweep(args.a0, args.orders, args.nt, args.precision, say=say)
    _table(recs, say)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(recs, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())

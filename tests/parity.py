"""Parity helpers: run the oracle on the same seeded inputs and compare.

Comparison protocol for the sub-cycling decision (several results can be
correct when psi0 sits within rounding of a threshold psi_max 4^k):
per-particle k traces are compared first; particles whose traces agree
must meet the tolerance directly; particles whose traces differ are
replayed by the oracle with the device's k sequence forced and must then
meet the tolerance, and every such flip must sit within rounding of a
threshold.
"""

from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O
from paper_2102_10983_amd import workloads as W


def oracle_fields(wl: W.Workload):
    table, M, shift = wl.table()
    return O.FieldSource(table=table, M=M, coeffs=W.shifted_coeffs(wl.lat, shift))


def oracle_params(wl: W.Workload, order=None, psi_max=None, k_max=8):
    return O.make_params(wl.ncells, wl.order if order is None else order, wl.dx, wl.dt,
                         wl.psi_max if psi_max is None else psi_max, wl.x_origin, k_max=k_max)


def oracle_yee_fields(wl: W.Workload, steps: int):
    """Standard PIC levels for the oracle: levels -order .. 0 sampled from
    the phase table, levels 1 .. steps - 1 from the FP64 Yee reference with
    the wave entering at node 0."""
    from oracle import yee_ref as Y
    table, M, shift = wl.table()
    aE, bE, cE, aB, bB, cB = (int(c) for c in W.shifted_coeffs(wl.lat, shift))
    p = wl.order
    i = np.arange(wl.ncells, dtype=np.int64)
    E = np.empty((steps + p, wl.ncells))
    B = np.empty((steps + p, wl.ncells))
    for j, m in enumerate(range(-p, 1)):
        E[j] = table[(aE * m + bE * i + cE) % M]
        B[j] = table[(aB * m + bB * i + cB) % M]
    if steps > 1:
        El, Bl = Y.advance_lattice(E[p], B[p], wl.dx, wl.dt, 1, steps - 1, table, aB, cB)
        E[p + 1:] = El
        B[p + 1:] = Bl
    return O.FieldSource(E=E, B=B, lev0=-p)


def oracle_run(wl, steps, idx=None, order=None, psi_max=None, trace=False, forced_k=None,
               k_old=None, threads=0, fields=None, k_max=8, state=None):
    idx = np.arange(wl.num) if idx is None else np.asarray(idx)
    x0, p0 = (wl.x0, wl.p0) if state is None else state
    st = O.State(x0[idx], p0[0][idx], p0[1][idx], p0[2][idx],
                 k_old=None if k_old is None else np.asarray(k_old)[idx])
    cnt = O.Counters()
    fs = oracle_fields(wl) if fields is None else fields
    kt, pt = O.push(oracle_params(wl, order, psi_max, k_max), fs, st, 0, steps,
                    trace=trace, psi_trace=trace, forced_k=forced_k, counters=cnt,
                    threads=threads)
    return st, cnt, kt, pt


def errors(gx, gpx, gpy, gpz, st: O.State, x0):
    """e_p = |p - p_ref| / max(|p_ref|, 1); e_x = |x - x_ref| / max(|x_ref - x0|, 2 pi)."""
    dp = np.sqrt((gpx - st.px) ** 2 + (gpy - st.py) ** 2 + (gpz - st.pz) ** 2)
    pref = np.sqrt(st.px ** 2 + st.py ** 2 + st.pz ** 2)
    e_p = dp / np.maximum(pref, 1.0)
    e_x = np.abs(gx - st.x) / np.maximum(np.abs(st.x - x0), 2 * math.pi)
    return e_p, e_x


def compare(wl, steps, gdiag, idx, tol, g_ktrace=None, order=None, psi_max=None,
            flip_rel=1e-9, fields=None, keep_each=False, k_max=8, state=None):
    """Compare device results (caller order, full arrays) on particles idx.

    flip_rel bounds how far from a threshold psi_max 4^k the first differing
    decision of a particle may lie (relative): rounding-level for the FP64
    path, the state difference the FP32 path is allowed for fp32c.
    Returns a dict of statistics (with keep_each, also the per-particle
    e_p under "e_p_each"); raises AssertionError on a violation."""
    idx = np.asarray(idx)
    st, cnt, kt, pt = oracle_run(wl, steps, idx, order=order, psi_max=psi_max,
                                 trace=g_ktrace is not None, fields=fields, k_max=k_max,
                                 state=state)
    gx, gpx, gpy, gpz = (gdiag[k][idx] for k in ("x", "px", "py", "pz"))
    out = {"n": len(idx), "flips": 0, "bitwise": 0}
    same = np.ones(len(idx), dtype=bool)
    if g_ktrace is not None:
        gk = g_ktrace[:, idx]
        same = np.all(gk == kt, axis=0)
        out["flips"] = int((~same).sum())
        if out["flips"]:
            # every flip must sit at a threshold: psi0 / psi_max within
            # rounding of 4^k at the first differing step
            worst = 0.0
            for c in np.nonzero(~same)[0]:
                s0 = int(np.argmax(gk[:, c] != kt[:, c]))
                r = pt[s0, c]
                kk = max(int(gk[s0, c]), int(kt[s0, c]))
                assert r > 0 and abs(r / 4.0 ** (kk - 1) - 1) < flip_rel, (c, s0, r, gk[s0, c],
                                                                           kt[s0, c])
                worst = max(worst, abs(r / 4.0 ** (kk - 1) - 1))
            out["worst_flip"] = worst
            fst, _, _, _ = oracle_run(wl, steps, idx[~same], order=order, psi_max=psi_max,
                                      forced_k=np.ascontiguousarray(gk[:, ~same]),
                                      fields=fields, k_max=k_max, state=state)
            st.x[~same], st.px[~same], st.py[~same], st.pz[~same] = fst.x, fst.px, fst.py, fst.pz
            st.status[~same] = fst.status
    e_p, e_x = errors(gx, gpx, gpy, gpz, st, (wl.x0 if state is None else state[0])[idx])
    if keep_each:
        out["e_p_each"] = e_p
    out["max_e_p"] = float(e_p.max()) if len(idx) else 0.0
    out["max_e_x"] = float(e_x.max()) if len(idx) else 0.0
    if len(idx):
        g_gam = np.sqrt(1.0 + gpx ** 2 + gpy ** 2 + gpz ** 2)
        out["max_e_gamma"] = float(np.max(np.abs(g_gam - st.gamma()) / st.gamma()))
        out["max_e_px"] = float(np.max(np.abs(gpx - st.px) / np.maximum(np.abs(st.px), 1.0)))
        out["p99_e_p"] = float(np.percentile(e_p, 99))
    out["bitwise"] = int(np.sum((gx == st.x) & (gpx == st.px) & (gpy == st.py) & (gpz == st.pz)))
    assert np.array_equal(gdiag["status"][idx], st.status), "status flags differ"
    assert out["max_e_p"] <= tol and out["max_e_x"] <= tol, out
    out["oracle_counters"] = cnt
    return out


def conditioning(wl, steps, idx, rel=1e-10, order=None, psi_max=None):
    """Sensitivity of the FP64 oracle's own trajectories: e_p between the
    oracle run from x0 and the run from x0 (1 + rel), per particle of idx.
    A path whose arithmetic acts on a trajectory like a perturbation of
    that size cannot be held closer than this to the oracle on that
    particle."""
    idx = np.asarray(idx)
    st, _, _, _ = oracle_run(wl, steps, idx, order=order, psi_max=psi_max)
    st2 = O.State(wl.x0[idx] * (1.0 + rel), wl.p0[0][idx], wl.p0[1][idx], wl.p0[2][idx])
    O.push(oracle_params(wl, order, psi_max), oracle_fields(wl), st2, 0, steps)
    e_p, _ = errors(st2.x, st2.px, st2.py, st2.pz, st, wl.x0[idx])
    return e_p

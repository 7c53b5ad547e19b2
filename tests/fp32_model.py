"""A float32 model of the FP32-compensated push, for error attribution.

Test infrastructure: a numpy model of the arithmetic a k = 0 step of the
compensated path performs, run step by step over many electrons, with the
sub-cycled steps handed to the FP64 oracle (forced to the model's k).  It
lets the precision of each part be switched on its own, so the source of
the error against the FP64 oracle can be shown on the CPU:

* ``decision``: "f64" takes the sub-cycling decision (Sec. IV, the Psi_max
  criterion) in FP64 from the FP64 value of the compensated momentum and B;
  "f32" takes it in float32 from the high words and a float32 B.
* ``transverse``: "boris" forms the y increment of the Boris update
  (Sec. III, Eqs. (p)..(gamman)) as 2h - a_x s, a difference of two terms
  of size |q E dt| that nearly cancel for an electron riding the wave;
  "split" forms the same quantity as 2c [(E - B) + B w] with E - B taken in
  FP64 before rounding and w = 1 - a_x / (gamma (1 + t^2)) written without
  cancellation (see ``_k0_step``); "kernel" is the operation sequence of
  the compensated kernel itself (``_k0_step_kernel``: float32 operations
  with explicit fused multiply-adds, c = q dt_p / 2 as a (hi, lo) pair, the
  low words of p folded into the first operations that use them).
* ``fields``: "f32" rounds E and B to float32 once per step; "f64" keeps
  them exact (an idealised reference for the attribution).
* ``exact``: names of quantities the "boris"/"split" steps keep in float64
  (attribution only): "c", "rot" (the rotation), "dpx", "dpy", "pos" (the
  position increment), "acc" (the accumulation), "p" (the whole momentum
  as the input of the step).
* ``rcp_ulps``: the float32 reciprocal and inverse square root carry this
  many ulps of (deterministic, sign-alternating) error, as hardware
  estimates without a Newton step may.

The position is carried as node index + float32 fraction + float32 carry
and moved by dt/dx (1 - (1 - |v_x|)) with 1 - |v_x| = (1 + p_y^2 + p_z^2) /
(gamma (gamma + |p_x|)); the momentum as float32 (hi, lo) pairs updated by
TwoSum.  Nothing here is imported by the product.
"""

from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O
from paper_2102_10983_amd import workloads as W

f32 = np.float32


def _two_sum(a, b):
    s = (a + b).astype(f32)
    bb = (s - a).astype(f32)
    e = ((a - (s - bb)) + (b - bb)).astype(f32)
    return s, e


def _comp_add(hi, lo, d):
    y = (d + lo).astype(f32)
    return _two_sum(hi, y)


def _split(v):
    hi = v.astype(f32)
    lo = (v - hi.astype(np.float64)).astype(f32)
    return hi, lo


def _rcp(x, ulps, tag):
    r = (1.0 / x.astype(np.float64)).astype(f32)
    if ulps:
        sgn = np.where(tag & 1, 1.0, -1.0).astype(f32)
        r = (r * (f32(1) + sgn * f32(ulps) * f32(2.0 ** -23))).astype(f32)
    return r


def _rsq(x, ulps, tag):
    r = (1.0 / np.sqrt(x.astype(np.float64))).astype(f32)
    if ulps:
        sgn = np.where(tag & 2, 1.0, -1.0).astype(f32)
        r = (r * (f32(1) + sgn * f32(ulps) * f32(2.0 ** -23))).astype(f32)
    return r


class Model:
    """Electrons of one workload advanced with the modelled arithmetic."""

    def __init__(self, wl: W.Workload, idx, *, decision="f64", transverse="split",
                 fields="f32", rcp_ulps=0, exact=(), c_split=True, lo_in=True,
                 pos64=False):
        self.wl = wl
        self.c_split, self.lo_in, self.pos64 = c_split, lo_in, pos64
        self.exact = set(exact)
        self.idx = np.asarray(idx)
        self.decision, self.transverse, self.fields = decision, transverse, fields
        self.rcp_ulps = int(rcp_ulps)
        table, M, shift = wl.table()
        self.table, self.M = table, int(M)
        self.co = tuple(int(c) for c in W.shifted_coeffs(wl.lat, shift))
        self.prm = O.make_params(wl.ncells, wl.order, wl.dx, wl.dt, wl.psi_max, wl.x_origin)
        self.fs = O.FieldSource(table=table, M=M, coeffs=self.co)
        _, self.LB = O.lagrange(wl.order, 0.5)
        n = len(self.idx)
        xi = (wl.x0[self.idx] - wl.x_origin) / wl.dx
        self.cell = np.floor(xi).astype(np.int64)
        self.fr, self.frc = _split(xi - self.cell)
        self.pxh, self.pxl = _split(wl.p0[0][self.idx])
        self.pyh, self.pyl = _split(wl.p0[1][self.idx])
        self.pzh, self.pzl = _split(wl.p0[2][self.idx])
        self.kold = np.full(n, -1, dtype=np.int64)
        self.status = np.zeros(n, dtype=np.uint8)
        dtdx = wl.dt / wl.dx
        self.dtdx_hi = f32(dtdx)
        self.dtdx_lo = f32(dtdx - float(self.dtdx_hi))
        self.tag = np.arange(n, dtype=np.int64)

    # fields on the lattice (the same values the oracle reads)
    def _E(self, m, i):
        aE, bE, cE = self.co[:3]
        return self.table[np.mod(aE * m + bE * i + cE, self.M)]

    def _B(self, m, i):
        aB, bB, cB = self.co[3:]
        return self.table[np.mod(aB * m + bB * i + cB, self.M)]

    def _p64(self):
        return (self.pxh.astype(np.float64) + self.pxl, self.pyh.astype(np.float64) + self.pyl,
                self.pzh.astype(np.float64) + self.pzl)

    def xi64(self):
        return self.cell + (self.fr.astype(np.float64) + self.frc.astype(np.float64))

    def step(self, n: int):
        wl, p = self.wl, self.wl.order
        xi = self.xi64()
        live = (self.status == 0) & (xi >= 0.5) & (xi < wl.ncells - 1)
        self.status[(self.status == 0) & ~live] = 1
        ib = np.where(live, np.floor(xi), 0).astype(np.int64)
        wb = xi - ib
        b0 = np.zeros(len(xi))
        b1 = np.zeros(len(xi))
        for j in range(p + 1):
            m = n - p + j
            b0 = b0 + self.LB[j] * self._B(m, ib)
            b1 = b1 + self.LB[j] * self._B(m, ib + 1)
        Bd = (1.0 - wb) * b0 + wb * b1
        c0 = 0.5 * wl.lat.dt * -1.0
        if self.decision == "f64":
            px, py, pz = self._p64()
            psi0 = np.abs(c0 * Bd) / np.sqrt(1.0 + ((px * px + py * py) + pz * pz))
            k = np.zeros(len(xi), dtype=np.int64)
            lim = np.full(len(xi), wl.psi_max)
            while True:
                up = (psi0 > lim) & (k < 8)
                if not up.any():
                    break
                k[up] += 1
                lim[up] *= 4.0
        else:
            p2 = ((self.pxh * self.pxh + self.pyh * self.pyh) + self.pzh * self.pzh).astype(f32)
            psi0 = (np.abs(f32(c0) * Bd.astype(f32)) *
                    _rsq((f32(1) + p2).astype(f32), self.rcp_ulps, self.tag)).astype(f32)
            k = np.zeros(len(xi), dtype=np.int64)
            lim = np.full(len(xi), f32(wl.psi_max), dtype=f32)
            while True:
                up = (psi0 > lim) & (k < 8)
                if not up.any():
                    break
                k[up] += 1
                lim[up] = (lim[up] * f32(4)).astype(f32)
        k[~live] = -1
        light = live & (k == 0)
        heavy = live & (k > 0)
        if light.any():
            if self.transverse == "kernel":
                self._k0_step_kernel(n, light, xi, Bd)
            else:
                self._k0_step(n, light, xi, Bd)
        if heavy.any():
            self._heavy_step(n, heavy, k)
        self.kold[live] = k[live]
        return k

    def _k0_step(self, n, sel, xi, Bd):
        wl = self.wl
        ex = self.exact

        def r(v, name):
            """Round to float32 unless `name` is kept exact (attribution)."""
            return np.asarray(v, dtype=np.float64) if name in ex else np.asarray(v).astype(f32)

        ko = np.where(self.kold[sel] < 0, 0, self.kold[sel])
        dtp = 0.5 * (np.ldexp(wl.dt, -2 * ko) + wl.dt)
        cf = r(0.5 * -1.0 * dtp, "c")
        x = xi[sel]
        uE = x - 0.5
        iE = np.floor(uE).astype(np.int64)
        wE = uE - iE
        E = (1.0 - wE) * self._E(n, iE) + wE * self._E(n, iE + 1)
        B = Bd[sel]
        fx = "fields" if self.fields == "f64" else "-"
        Ef, Bf = r(E, fx), r(B, fx)
        tag = self.tag[sel]
        u = self.rcp_ulps

        def rcp(v, name):
            return 1.0 / np.asarray(v, dtype=np.float64) if name in ex else _rcp(v, u, tag)

        def rsq(v, name):
            return (1.0 / np.sqrt(np.asarray(v, dtype=np.float64)) if name in ex
                    else _rsq(v, u, tag))

        pxh, pxl = self.pxh[sel], self.pxl[sel]
        pyh, pyl = self.pyh[sel], self.pyl[sel]
        pzh = self.pzh[sel]
        if "p" in ex:             # the whole momentum, not the high word
            mx0 = pxh.astype(np.float64) + pxl
            my0 = pyh.astype(np.float64) + pyl
        else:
            mx0, my0 = pxh, pyh
        h = r(cf * Ef, "rot")
        mx, my, mz = mx0, r(my0 + h, "rot"), pzh
        gg = r(1.0 + ((mx * mx + my * my) + mz * mz), "rot")
        ig = rsq(gg, "rot")
        t = r((cf * Bf) * ig, "rot")
        opt = r(1.0 + t * t, "rot")
        sz = r((2.0 * t) * rcp(opt, "rot"), "rot")
        ax = r(mx + my * t, "rot")
        ay = r(my - mx * t, "rot")
        dpx = r(ay * sz, "dpx")
        if self.transverse == "boris":
            dpy = r((h + h) - ax * sz, "dpy")
        else:
            D = r(E - B, fx)
            g = r(gg * ig, "rot")                       # gamma of m
            fwd = mx >= 0
            num_f = r((1.0 + (my * my + mz * mz)) * rcp(r(g + mx, "dpy"), "dpy")
                      + t * (cf * Bf - my), "dpy")
            num_b = r(g * opt - ax, "dpy")
            num = np.where(fwd, num_f, num_b)
            w = r(num * rcp(r(g * opt, "dpy"), "dpy"), "dpy")
            dpy = r((cf + cf) * (D + Bf * w), "dpy")
        if "acc" in ex:           # exact accumulation (FP64 sum, then split)
            self.pxh[sel], self.pxl[sel] = _split(pxh.astype(np.float64) + pxl + dpx)
            self.pyh[sel], self.pyl[sel] = _split(pyh.astype(np.float64) + pyl + dpy)
        else:
            self.pxh[sel], self.pxl[sel] = _comp_add(pxh, pxl, dpx.astype(f32))
            self.pyh[sel], self.pyl[sel] = _comp_add(pyh, pyl, dpy.astype(f32))
        # position: node units, cell + fraction + carry
        if "p" in ex:
            qx = self.pxh[sel].astype(np.float64) + self.pxl[sel]
            qy = self.pyh[sel].astype(np.float64) + self.pyl[sel]
        else:
            qx, qy = self.pxh[sel], self.pyh[sel]
        qz = pzh
        q2 = r(qy * qy + qz * qz, "pos")
        g2 = r(np.sqrt(r(1.0 + (qx * qx + q2), "pos")), "pos")
        omv = r((1.0 + q2) * rcp(r(g2 * (g2 + np.abs(qx)), "pos"), "pos"), "pos")
        sgn = np.where(qx < 0, -1.0, 1.0)
        if "pos" in ex:
            xi_new = self.xi64()[sel] + sgn * (wl.dt / wl.dx) * (1.0 - omv)
            c = np.floor(xi_new).astype(np.int64)
            self.cell[sel] = c
            self.fr[sel], self.frc[sel] = _split(xi_new - c)
            return
        sgn = sgn.astype(f32)
        omv = omv.astype(f32)
        fr, frc = self.fr[sel], self.frc[sel]
        s1, e1 = _two_sum(fr, (sgn * self.dtdx_hi).astype(f32))
        y = (((sgn * (self.dtdx_lo - self.dtdx_hi * omv)) + e1) + frc).astype(f32)
        s2, e2 = _two_sum(s1, y)
        adj = np.where(s2 >= 1, f32(-1), np.where(s2 < 0, f32(1), f32(0))).astype(f32)
        self.cell[sel] -= adj.astype(np.int64)
        fr2, e3 = _two_sum(s2, adj)
        self.fr[sel] = fr2
        self.frc[sel] = (e2 + e3).astype(f32)

    def _k0_step_kernel(self, n, sel, xi, Bd):
        """The k = 0 step as the compensated kernel computes it: float32
        operations (fma = one rounding), the low words of p folded into the
        first operation that uses them, c = q dt_p / 2 as a (hi, lo) pair,
        E - B formed in FP64 before rounding, and the position moved by
        dt/dx minus dt/dx (1 - |v_x|) with 1 - |v_x| in FP64 when
        ``pos64`` is set."""
        wl = self.wl

        def fma(a, b, c):
            return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
                    + np.asarray(c, np.float64)).astype(f32)

        def mul(a, b):
            return (np.asarray(a, np.float64) * np.asarray(b, np.float64)).astype(f32)

        def add(a, b):
            return (np.asarray(a, np.float64) + np.asarray(b, np.float64)).astype(f32)

        tag = self.tag[sel]
        u = self.rcp_ulps
        ko = np.where(self.kold[sel] < 0, 0, self.kold[sel])
        c64 = 0.5 * -1.0 * (0.5 * (np.ldexp(wl.dt, -2 * ko) + wl.dt))
        ch = c64.astype(f32)
        cl = (c64 - ch).astype(f32) if self.c_split else np.zeros_like(ch)
        x = xi[sel]
        uE = x - 0.5
        iE = np.floor(uE).astype(np.int64)
        wE = uE - iE
        E = (1.0 - wE) * self._E(n, iE) + wE * self._E(n, iE + 1)
        B = Bd[sel]
        Ef, Bf, Df = E.astype(f32), B.astype(f32), (E - B).astype(f32)
        pxh, pxl = self.pxh[sel], self.pxl[sel]
        pyh, pyl = self.pyh[sel], self.pyl[sel]
        pzh = self.pzh[sel]
        lo = self.lo_in
        h = fma(cl, Ef, mul(ch, Ef))
        my = add(add(pyh, h), pyl) if lo else add(pyh, h)
        onepz = fma(pzh, pzh, f32(1))
        gg = fma(my, my, onepz)
        gg = fma(pxh, pxh, gg)
        if lo:
            gg = fma(add(pxh, pxh), pxl, gg)
        ig = _rsq(gg, u, tag)
        cB = fma(cl, Bf, mul(ch, Bf))
        t = mul(cB, ig)
        opt = fma(t, t, f32(1))
        sz = mul(add(t, t), _rcp(opt, u, tag))
        ax = fma(my, t, pxh)
        if lo:
            ax = add(ax, pxl)
        ay = fma(-pxh, t, my)
        dpx = mul(ay, sz)
        g = mul(gg, ig)
        fwd = pxh >= 0
        q1 = fma(my, my, onepz)
        num_f = fma(t, add(cB, -my), mul(q1, _rcp(add(g, pxh), u, tag)))
        num_b = fma(g, opt, -ax)
        num = np.where(fwd, num_f, num_b)
        w = mul(num, _rcp(mul(g, opt), u, tag))
        dpy = mul(add(ch, ch), fma(Bf, w, Df))
        if self.c_split:
            dpy = fma(add(cl, cl), fma(Bf, w, Df), dpy)
        self.pxh[sel], self.pxl[sel] = _comp_add(pxh, pxl, dpx)
        self.pyh[sel], self.pyl[sel] = _comp_add(pyh, pyl, dpy)
        qxh, qxl = self.pxh[sel], self.pxl[sel]
        qyh, qyl = self.pyh[sel], self.pyl[sel]
        if self.pos64:
            qx = qxh.astype(np.float64) + qxl
            qy = qyh.astype(np.float64) + qyl
            qz = pzh.astype(np.float64)
            q2 = qy * qy + qz * qz
            g2 = np.sqrt(1.0 + (qx * qx + q2))
            omv64 = (1.0 + q2) / (g2 * (g2 + np.abs(qx)))
            omv = omv64.astype(f32)
            omv_lo = (omv64 - omv).astype(f32)
        else:
            q2 = fma(qyh, qyh, mul(pzh, pzh))
            if lo:
                q2 = fma(add(qyh, qyh), qyl, q2)
            gg2 = add(f32(1), fma(qxh, qxh, q2))
            if lo:
                gg2 = fma(add(qxh, qxh), qxl, gg2)
            g2 = np.sqrt(gg2.astype(np.float64)).astype(f32)
            ax2 = np.abs(qxh)
            omv = mul(add(f32(1), q2), _rcp(mul(g2, add(g2, ax2)), u, tag))
            omv_lo = np.zeros_like(omv)
        sgn = np.where(qxh < 0, f32(-1), f32(1)).astype(f32)
        fr, frc = self.fr[sel], self.frc[sel]
        s1, e1 = _two_sum(fr, mul(sgn, self.dtdx_hi))
        corr = fma(-self.dtdx_hi, omv, self.dtdx_lo)
        corr = fma(-self.dtdx_hi, omv_lo, corr)
        y = add(add(mul(sgn, corr), e1), frc)
        s2, e2 = _two_sum(s1, y)
        adj = np.where(s2 >= 1, f32(-1), np.where(s2 < 0, f32(1), f32(0))).astype(f32)
        self.cell[sel] -= adj.astype(np.int64)
        fr2, e3 = _two_sum(s2, adj)
        self.fr[sel] = fr2
        self.frc[sel] = add(e2, e3)

    def _heavy_step(self, n, sel, k):
        wl = self.wl
        px, py, pz = self._p64()
        x = wl.x_origin + self.xi64()[sel] * wl.dx
        st = O.State(x, px[sel], py[sel], pz[sel], k_old=self.kold[sel].astype(np.int8))
        O.push(self.prm, self.fs, st, n, 1, forced_k=k[sel][None, :].astype(np.int8))
        xi = (st.x - wl.x_origin) / wl.dx
        c = np.floor(xi).astype(np.int64)
        self.cell[sel] = c
        self.fr[sel], self.frc[sel] = _split(xi - c)
        self.pxh[sel], self.pxl[sel] = _split(st.px)
        self.pyh[sel], self.pyl[sel] = _split(st.py)
        self.pzh[sel], self.pzl[sel] = _split(st.pz)
        self.status[sel] = st.status

    def run(self, steps: int):
        kt = np.empty((steps, len(self.idx)), dtype=np.int8)
        for n in range(steps):
            kt[n] = self.step(n)
        return kt

    def state(self):
        px, py, pz = self._p64()
        x = self.wl.x_origin + self.xi64() * self.wl.dx
        return {"x": x, "px": px, "py": py, "pz": pz, "status": self.status.copy()}


def errors_vs_oracle(wl: W.Workload, idx, model_state, model_kt, steps: int,
                     flip_rel: float):
    """Errors of the model against the FP64 oracle under the k-flip
    protocol; returns a dict (max e_p, p99 e_p, max e_x, max e_gamma, flips,
    largest |psi0 / threshold - 1| among the flips)."""
    idx = np.asarray(idx)
    prm = O.make_params(wl.ncells, wl.order, wl.dx, wl.dt, wl.psi_max, wl.x_origin)
    table, M, shift = wl.table()
    fs = O.FieldSource(table=table, M=M, coeffs=W.shifted_coeffs(wl.lat, shift))
    st = O.State(wl.x0[idx], wl.p0[0][idx], wl.p0[1][idx], wl.p0[2][idx])
    kt, pt = O.push(prm, fs, st, 0, steps, trace=True, psi_trace=True)
    same = np.all(model_kt == kt, axis=0)
    worst_flip = 0.0
    for c in np.nonzero(~same)[0]:
        s0 = int(np.argmax(model_kt[:, c] != kt[:, c]))
        kk = max(int(model_kt[s0, c]), int(kt[s0, c]))
        worst_flip = max(worst_flip, abs(pt[s0, c] / 4.0 ** (kk - 1) - 1.0))
    if (~same).any():
        fst = O.State(wl.x0[idx][~same], wl.p0[0][idx][~same], wl.p0[1][idx][~same],
                      wl.p0[2][idx][~same])
        O.push(prm, fs, fst, 0, steps, forced_k=np.ascontiguousarray(model_kt[:, ~same]))
        st.x[~same], st.px[~same], st.py[~same], st.pz[~same] = fst.x, fst.px, fst.py, fst.pz
        st.status[~same] = fst.status
    g = model_state
    dp = np.sqrt((g["px"] - st.px) ** 2 + (g["py"] - st.py) ** 2 + (g["pz"] - st.pz) ** 2)
    pref = np.sqrt(st.px ** 2 + st.py ** 2 + st.pz ** 2)
    e_p = dp / np.maximum(pref, 1.0)
    e_x = np.abs(g["x"] - st.x) / np.maximum(np.abs(st.x - wl.x0[idx]), 2 * math.pi)
    gam = np.sqrt(1.0 + g["px"] ** 2 + g["py"] ** 2 + g["pz"] ** 2)
    e_g = np.abs(gam - st.gamma()) / st.gamma()
    return {"max_e_p": float(e_p.max()), "p99_e_p": float(np.percentile(e_p, 99)),
            "max_e_x": float(e_x.max()), "max_e_gamma": float(e_g.max()),
            "flips": int((~same).sum()), "worst_flip": worst_flip,
            "flips_within": bool(worst_flip < flip_rel),
            "status_equal": bool(np.array_equal(g["status"], st.status))}

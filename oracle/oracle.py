"""ctypes binding of the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
KHIST = 16
MAX_ORDER = 7


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB_PATH,
               os.path.join(HERE, "oracle.c"), "-lm"]
        subprocess.check_call(cmd)
    return LIB_PATH


class Params(C.Structure):
    _fields_ = [("ncells", C.c_int32), ("order", C.c_int32), ("k_max", C.c_int32),
                ("pad_", C.c_int32), ("x_origin", C.c_double), ("dx", C.c_double),
                ("dt", C.c_double), ("qm", C.c_double), ("psi_max", C.c_double)]


class Fields(C.Structure):
    _fields_ = [("mode", C.c_int32), ("nlev", C.c_int32), ("lev0", C.c_int64),
                ("E", C.c_void_p), ("B", C.c_void_p), ("table", C.c_void_p),
                ("M", C.c_int64), ("aE", C.c_int64), ("bE", C.c_int64), ("cE", C.c_int64),
                ("aB", C.c_int64), ("bB", C.c_int64), ("cB", C.c_int64),
                ("atab", C.c_void_p)]


class Counters(C.Structure):
    _fields_ = [("steps", C.c_uint64), ("sub_steps", C.c_uint64), ("n_star", C.c_uint64),
                ("clamps", C.c_uint64), ("lost", C.c_uint64),
                ("steps_by_k", C.c_uint64 * KHIST), ("sub_steps_by_k", C.c_uint64 * KHIST)]

    def as_dict(self):
        return {"steps": self.steps, "sub_steps": self.sub_steps, "n_star": self.n_star,
                "clamps": self.clamps, "lost": self.lost,
                "steps_by_k": list(self.steps_by_k), "sub_steps_by_k": list(self.sub_steps_by_k)}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_lagrange.argtypes = [C.c_int32, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_lagrange.restype = C.c_int
        L.orc_gather.argtypes = [C.POINTER(Params), C.POINTER(Fields), C.c_int32, C.c_int64,
                                 C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.orc_gather.restype = C.c_int
        L.orc_decide_k.argtypes = [C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_int32)]
        L.orc_decide_k.restype = C.c_int32
        L.orc_boris.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]
        L.orc_boris.restype = None
        L.orc_push.argtypes = [C.POINTER(Params), C.POINTER(Fields), C.c_int64,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                               C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_void_p, C.POINTER(Counters), C.c_int32]
        L.orc_push.restype = C.c_int
        L.orc_max_threads.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def lagrange(order: int, s: float):
    LE = np.zeros(order + 1)
    LB = np.zeros(order + 1)
    if lib().orc_lagrange(order, s, _ptr(LE), _ptr(LB)) != 0:
        raise ValueError("bad order")
    return LE, LB


def decide_k(psi0: float, psi_max: float, k_max: int):
    cl = C.c_int32(0)
    k = lib().orc_decide_k(psi0, psi_max, k_max, C.byref(cl))
    return k, bool(cl.value)


def boris(qm, dtp, E, B, p):
    px, py, pz = (C.c_double(float(v)) for v in p)
    lib().orc_boris(qm, dtp, E, B, C.byref(px), C.byref(py), C.byref(pz))
    return np.array([px.value, py.value, pz.value])


class FieldSource:
    """Explicit levels (E[L, ncells], B[L, ncells] from level lev0) or a
    lattice table (F = table[(a n + b i + c) mod M])."""

    def __init__(self, *, E=None, B=None, lev0=0, table=None, M=0, coeffs=None, atab=None):
        self.s = Fields()
        if table is not None:
            self._keep = (np.ascontiguousarray(table, dtype=np.float64),)
            self.s.mode = 1
            self.s.table = self._keep[0].ctypes.data
            if atab is not None:
                at = np.ascontiguousarray(atab, dtype=np.float64)
                assert at.shape == self._keep[0].shape
                self._keep = self._keep + (at,)
                self.s.atab = at.ctypes.data
            self.s.M = int(M)
            (self.s.aE, self.s.bE, self.s.cE, self.s.aB, self.s.bB, self.s.cB) = (
                int(c) for c in coeffs)
        else:
            E = np.ascontiguousarray(E, dtype=np.float64)
            B = np.ascontiguousarray(B, dtype=np.float64)
            assert E.shape == B.shape and E.ndim == 2
            self._keep = (E, B)
            self.s.mode = 0
            self.s.E = E.ctypes.data
            self.s.B = B.ctypes.data
            self.s.lev0 = int(lev0)
            self.s.nlev = E.shape[0]


def make_params(ncells, order, dx, dt, psi_max, x_origin=0.0, qm=-1.0, k_max=8):
    return Params(ncells=ncells, order=order, k_max=k_max, pad_=0, x_origin=x_origin,
                  dx=dx, dt=dt, qm=qm, psi_max=psi_max)


def gather(prm: Params, fs: FieldSource, which: int, n: int, s: float, x: float):
    out = C.c_double(0.0)
    rc = lib().orc_gather(C.byref(prm), C.byref(fs.s), which, n, s, x, C.byref(out))
    if rc != 0:
        raise ValueError(f"orc_gather failed ({rc})")
    return out.value


class State:
    """Particle state arrays owned by the caller (numpy, float64)."""

    def __init__(self, x, px=None, py=None, pz=None, k_old=None):
        num = len(x)
        z = np.zeros(num)
        self.x = np.array(x, dtype=np.float64)
        self.px = np.array(z if px is None else px, dtype=np.float64)
        self.py = np.array(z if py is None else py, dtype=np.float64)
        self.pz = np.array(z if pz is None else pz, dtype=np.float64)
        self.k_old = (np.full(num, -1, dtype=np.int8) if k_old is None
                      else np.array(k_old, dtype=np.int8))
        self.status = np.zeros(num, dtype=np.uint8)

    @property
    def num(self):
        return len(self.x)

    def gamma(self):
        return np.sqrt(1.0 + self.px ** 2 + self.py ** 2 + self.pz ** 2)

    def copy(self):
        c = State(self.x, self.px, self.py, self.pz, self.k_old)
        c.status = self.status.copy()
        return c


def push(prm: Params, fs: FieldSource, st: State, n0: int, nsteps: int, *,
         forced_k=None, trace=False, psi_trace=False, counters: Counters | None = None,
         threads: int = 0, work=None, werr=None, r0=None, rmax=None, gmax=None,
         ai=None, emax=None):
    """Advance the state in place; returns (k_trace, psi_trace) arrays or None.
    work, werr: float64 arrays of st.num updated in place (App. B energy
    accounting); r0, rmax: the dephasing error of Eq. (R error) against r0,
    running maximum kept in rmax; gmax: running maximum of gamma; ai, emax:
    the energy error of Eq. (gamma error), running maximum kept in emax
    (needs a field source with atab; see orc_push)."""
    if r0 is not None:
        r0 = np.ascontiguousarray(r0, dtype=np.float64)
    if ai is not None:
        ai = np.ascontiguousarray(ai, dtype=np.float64)
    for a in (work, werr, rmax, gmax, emax):
        if a is not None:
            assert a.dtype == np.float64 and a.shape == (st.num,) and a.flags.c_contiguous
    kt = np.empty((nsteps, st.num), dtype=np.int8) if trace else None
    pt = np.empty((nsteps, st.num), dtype=np.float64) if psi_trace else None
    fk = None if forced_k is None else np.ascontiguousarray(forced_k, dtype=np.int8)
    if fk is not None:
        assert fk.shape == (nsteps, st.num)
    cnt = counters if counters is not None else Counters()
    rc = lib().orc_push(C.byref(prm), C.byref(fs.s), st.num, _ptr(st.x), _ptr(st.px),
                        _ptr(st.py), _ptr(st.pz), _ptr(st.k_old), _ptr(st.status),
                        n0, nsteps, _ptr(fk), _ptr(kt), _ptr(pt), _ptr(work), _ptr(werr),
                        _ptr(r0), _ptr(rmax), _ptr(gmax), _ptr(ai), _ptr(emax),
                        C.byref(cnt), threads)
    if rc != 0:
        raise ValueError(f"orc_push failed ({rc})")
    return kt, pt


def dephasing_R(px, py, pz):
    """R = gamma - p_x (Sec. V), gamma = sqrt(1 + ((p_x^2 + p_y^2) + p_z^2))."""
    px = np.asarray(px, dtype=np.float64)
    py = np.asarray(py, dtype=np.float64)
    pz = np.asarray(pz, dtype=np.float64)
    return np.sqrt(1.0 + ((px * px + py * py) + pz * pz)) - px


def push_diagnostics(prm: Params, fs: FieldSource, st: State, n0: int, nsteps: int, *,
                     forced_k=None, counters: Counters | None = None, threads: int = 0,
                     gmax=None):
    """push() one step at a time, recording after every completed step of a
    live particle the dephasing error |R - R0| / R0 of Eq. (R error), R0
    being R of the state passed in, and the energy accounting of App. B.
    Returns (R0, running max of the dephasing error, work since the start,
    largest per-step |kinetic energy change - work|, k trace [nsteps, num]).
    gmax: optional float64 array of st.num, the running maximum of gamma,
    updated in place (see orc_push)."""
    R0 = dephasing_R(st.px, st.py, st.pz)
    rmax = np.zeros(st.num)
    work = np.zeros(st.num)
    werr = np.zeros(st.num)
    kt = np.empty((nsteps, st.num), dtype=np.int8)
    cnt = counters if counters is not None else Counters()
    for c in range(nsteps):
        live_before = st.status == 0
        fk = None if forced_k is None else np.ascontiguousarray(forced_k[c:c + 1])
        k1, _ = push(prm, fs, st, n0 + c, 1, forced_k=fk, trace=True, counters=cnt,
                     threads=threads, work=work, werr=werr, gmax=gmax)
        kt[c] = k1[0]
        done = live_before & (st.status == 0)
        d = np.abs(dephasing_R(st.px, st.py, st.pz) - R0) / R0
        rmax = np.where(done & (d > rmax), d, rmax)
    return R0, rmax, work, werr, kt


def max_threads() -> int:
    return int(lib().orc_max_threads())

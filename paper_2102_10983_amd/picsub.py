"""Python binding of libpicsub (the C ABI declared in include/picsub.h).

Argument marshalling only: every step of the push runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: if libpicsub.so is missing or no GPU is present, the calls raise.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpicsub.so")

PIC_KHIST = 16
PIC_K_MAX_LIMIT = 8
STATUS = {0: "PIC_OK", 1: "PIC_E_ARG", 2: "PIC_E_DEVICE", 3: "PIC_E_NOMEM",
          4: "PIC_E_LEVEL", 5: "PIC_E_STATE", 6: "PIC_E_NUMERIC"}
PRECISION = {"fp64": 0, "fp32c": 1, "fp64fast": 2}
BINNING = {"none": 0, "ballot": 1, "learned": 2}
MEM_HOST, MEM_DEVICE = 0, 1

# every symbol the header declares
EXPORTS = ("pic_create", "pic_destroy", "pic_last_error", "pic_particles_set",
           "pic_fields_load", "pic_fields_load_lattice", "pic_push_subcycled",
           "pic_ktrace_set", "pic_diag", "pic_diag_noalloc", "pic_diag_r", "pic_strict_set",
           "pic_grid_shift",
           "pic_counters_reset",
           "pic_batch_create",
           "pic_fields_load_r", "pic_fields_load_lattice_r", "pic_source_set", "pic_advance",
           "pic_run_level", "pic_graph_capture", "pic_graph_launch", "pic_graph_release",
           "pic_run_counters", "pic_tune_set", "pic_tune_get", "pic_autotune",
           "pic_group_count", "pic_order_set", "pic_features", "pic_mlp_forward",
           "pic_mlp_grad", "pic_mlp_adam", "pic_prebin", "pic_state_export",
           "pic_state_import", "pic_fields_yee", "pic_fields_yee_r", "pic_fields_read",
           "pic_fields_read_r", "pic_diag_track", "pic_dephasing_read",
           "pic_energy_read", "pic_gamma_max_read", "pic_fma_probe", "pic_ktrace_load",
           "pic_gamma_error_lattice", "pic_gamma_error_start", "pic_gamma_error_read",
           "pic_predictor_set", "pic_autotune_forget")

MLP_FEATURES = 8
MLP_HIDDEN = 64
MLP_NPARAM = 4801
NO_LEVEL = -(1 << 63)


class PicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("ncells", C.c_int32), ("order", C.c_int32), ("ring_depth", C.c_int32),
                ("k_max", C.c_int32), ("precision", C.c_int32), ("binning", C.c_int32),
                ("x_origin", C.c_double), ("dx", C.c_double), ("dt", C.c_double),
                ("qm", C.c_double), ("psi_max", C.c_double)]


class Counters(C.Structure):
    _fields_ = [("steps", C.c_uint64), ("sub_steps", C.c_uint64), ("n_star", C.c_uint64),
                ("clamps", C.c_uint64), ("lost", C.c_uint64),
                ("steps_by_k", C.c_uint64 * PIC_KHIST),
                ("sub_steps_by_k", C.c_uint64 * PIC_KHIST), ("rebins", C.c_uint64)]

    def as_dict(self):
        return {"steps": self.steps, "sub_steps": self.sub_steps, "n_star": self.n_star,
                "clamps": self.clamps, "lost": self.lost,
                "steps_by_k": list(self.steps_by_k),
                "sub_steps_by_k": list(self.sub_steps_by_k), "rebins": self.rebins}


class Tune(C.Structure):
    _fields_ = [("waves_per_group", C.c_int32), ("tile", C.c_int32), ("binning", C.c_int32),
                ("sort_sub", C.c_int32), ("occupancy", C.c_int32)]

    def as_dict(self):
        return {"waves_per_group": self.waves_per_group, "tile": self.tile,
                "binning": {v: k for k, v in BINNING.items()}[self.binning],
                "sort_sub": self.sort_sub, "occupancy": self.occupancy}


_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load libpicsub.so and declare the signatures (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pic_create": ([C.POINTER(Params), i64, vp, C.POINTER(vp)], C.c_int),
        "pic_destroy": ([vp], C.c_int),
        "pic_last_error": ([vp], C.c_char_p),
        "pic_particles_set": ([vp, C.c_int, vp, vp, vp, vp, vp], C.c_int),
        "pic_fields_load": ([vp, i64, C.c_int, vp, vp], C.c_int),
        "pic_fields_load_lattice": ([vp, i64, i32, vp, i64, i64, i64, i64, i64, i64, i64],
                                    C.c_int),
        "pic_push_subcycled": ([vp, i64, i32], C.c_int),
        "pic_ktrace_set": ([vp, vp, i64, i32, i64, i64], C.c_int),
        "pic_diag": ([vp, C.c_int, vp, vp, vp, vp, vp, vp, vp, C.POINTER(Counters)], C.c_int),
        "pic_diag_noalloc": ([vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(Counters)], C.c_int),
        "pic_diag_r": ([vp, i32, C.c_int, vp, vp, vp, vp, vp, vp, vp, C.POINTER(Counters)],
                       C.c_int),
        "pic_strict_set": ([vp, i32], C.c_int),
        "pic_grid_shift": ([vp, i32, i64, C.POINTER(dbl)], C.c_int),
        "pic_counters_reset": ([vp], C.c_int),
        "pic_batch_create": ([vp, vp, i32, vp, C.POINTER(vp)], C.c_int),
        "pic_fields_load_r": ([vp, i32, i64, C.c_int, vp, vp], C.c_int),
        "pic_fields_load_lattice_r": ([vp, i32, i64, i32, vp, i64, i64, i64, i64, i64, i64,
                                       i64], C.c_int),
        "pic_source_set": ([vp, i32, i64, i64, vp, i64, i64, i64, i64, i64, i64, i64], C.c_int),
        "pic_advance": ([vp, i32], C.c_int),
        "pic_run_level": ([vp, i32, C.POINTER(i64)], C.c_int),
        "pic_graph_capture": ([vp, i32, i32], C.c_int),
        "pic_graph_launch": ([vp], C.c_int),
        "pic_graph_release": ([vp], C.c_int),
        "pic_run_counters": ([vp, i32, C.POINTER(Counters)], C.c_int),
        "pic_tune_set": ([vp, C.POINTER(Tune)], C.c_int),
        "pic_tune_get": ([vp, C.POINTER(Tune)], C.c_int),
        "pic_autotune": ([vp, i32, i32, C.POINTER(Tune), C.POINTER(dbl)], C.c_int),
        "pic_group_count": ([vp], i32),
        "pic_order_set": ([vp, vp, C.c_int], C.c_int),
        "pic_features": ([vp, i64, vp, vp], C.c_int),
        "pic_mlp_forward": ([vp, vp, vp, vp, i64, vp], C.c_int),
        "pic_mlp_grad": ([vp, vp, vp, vp, i64, C.c_float, vp, vp, vp], C.c_int),
        "pic_mlp_adam": ([vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, i32,
                          vp], C.c_int),
        "pic_prebin": ([vp, vp, i32, C.c_float, i32], C.c_int),
        "pic_state_export": ([vp, vp, C.POINTER(C.c_size_t)], C.c_int),
        "pic_state_import": ([vp, vp, C.c_size_t, vp], C.c_int),
        "pic_fields_yee": ([vp, i64, i32, vp, i64, i64, i64], C.c_int),
        "pic_fields_yee_r": ([vp, i32, i64, i32, vp, i64, i64, i64], C.c_int),
        "pic_fields_read": ([vp, i64, C.c_int, vp, vp], C.c_int),
        "pic_fields_read_r": ([vp, i32, i64, C.c_int, vp, vp], C.c_int),
        "pic_diag_track": ([vp, i32], C.c_int),
        "pic_energy_read": ([vp, C.c_int, vp, vp], C.c_int),
        "pic_gamma_max_read": ([vp, C.c_int, vp], C.c_int),
        "pic_gamma_error_lattice": ([vp, i32, vp, C.c_int64, C.c_int64, C.c_int64, C.c_int64],
                                    C.c_int),
        "pic_gamma_error_start": ([vp, C.c_int, vp], C.c_int),
        "pic_gamma_error_read": ([vp, C.c_int, vp], C.c_int),
        "pic_fma_probe": ([vp, i32, C.c_int64, vp], C.c_int),
        "pic_ktrace_load": ([vp, i32, C.c_int64, vp, vp], C.c_int),
        "pic_predictor_set": ([vp, vp, vp, vp, C.c_float, i32], C.c_int),
        "pic_autotune_forget": ([], C.c_int),
        "pic_dephasing_read": ([vp, C.c_int, vp, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if path == LIB_PATH:
        _lib = L
    return L


def autotune_forget():
    """Clear the process-wide memory of autotuned launch shapes."""
    st = load_library().pic_autotune_forget()
    if st != 0:
        raise PicError(st, "pic_autotune_forget failed")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libpicsub needs a ROCm GPU; none is visible")
    return torch


def _dev_ptr(t, dtype, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return t.data_ptr()


def make_params(*, ncells: int, order: int, dx: float, dt: float, psi_max: float,
                x_origin: float = 0.0, qm: float = -1.0, k_max: int = 8,
                ring_depth: int | None = None, precision: str = "fp64",
                binning: str = "none") -> Params:
    return Params(ncells=ncells, order=order, ring_depth=int(ring_depth or (order + 1)),
                  k_max=k_max, precision=PRECISION[precision], binning=BINNING[binning],
                  x_origin=x_origin, dx=dx, dt=dt, qm=qm, psi_max=psi_max)


class Pusher:
    """One context of the C ABI: a batch of runs (one run by default), each
    with its particles and field ring, on one stream.

    Pusher(num=..., ncells=..., ...) builds a one-run context;
    Pusher(runs=[(num, Params), ...]) a batch."""

    def __init__(self, *, num: int | None = None, runs=None, stream=None, **kw):
        torch = _torch()
        self._lib = load_library()
        if runs is None:
            runs = [(int(num), make_params(**kw))]
        self.nruns = len(runs)
        self.nums = [int(n) for n, _ in runs]
        self.num = sum(self.nums)
        self.offsets = np.concatenate([[0], np.cumsum(self.nums)]).astype(np.int64)
        self.params = [p for _, p in runs]
        self.prm = self.params[0]
        self.order = int(self.prm.order)
        self.ring_depth = int(self.prm.ring_depth)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (Params * self.nruns)(*self.params)
        counts = (C.c_int64 * self.nruns)(*self.nums)
        self._ctx = C.c_void_p()
        st = self._lib.pic_batch_create(arr, counts, self.nruns,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx))
        if st != 0:
            msg = self._err()
            if self._ctx:
                self._lib.pic_destroy(self._ctx)
                self._ctx = C.c_void_p()
            raise PicError(st, msg)
        self._keep = []
        self._sources = {}

    # -- helpers ---------------------------------------------------------
    def _err(self) -> str:
        if not self._ctx:
            return "context creation failed"
        m = self._lib.pic_last_error(self._ctx)
        return m.decode() if m else ""

    def _check(self, st: int):
        if st != 0:
            raise PicError(st, self._err())

    def close(self):
        if self._ctx:
            self._lib.pic_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls -----------------------------------------------------------
    def particles_set(self, x, px, py, pz, k_old=None):
        """Device tensors (float64, int8) or host numpy arrays."""
        torch = _torch()
        n = self.num
        if isinstance(x, torch.Tensor):
            ptrs = [_dev_ptr(a, torch.float64, n) for a in (x, px, py, pz)]
            kp = None if k_old is None else _dev_ptr(k_old, torch.int8, n)
            self._check(self._lib.pic_particles_set(self._ctx, MEM_DEVICE, *ptrs, kp))
        else:
            arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, px, py, pz)]
            for a in arrs:
                if a.size != n:
                    raise ValueError("wrong particle count")
            ka = None if k_old is None else np.ascontiguousarray(k_old, dtype=np.int8)
            self._check(self._lib.pic_particles_set(
                self._ctx, MEM_HOST, *[a.ctypes.data for a in arrs],
                None if ka is None else ka.ctypes.data))

    def fields_load(self, n: int, Ey, Bz):
        torch = _torch()
        if isinstance(Ey, torch.Tensor):
            nc = self.prm.ncells
            self._check(self._lib.pic_fields_load(self._ctx, n, MEM_DEVICE,
                                                  _dev_ptr(Ey, torch.float64, nc),
                                                  _dev_ptr(Bz, torch.float64, nc)))
        else:
            E = np.ascontiguousarray(Ey, dtype=np.float64)
            B = np.ascontiguousarray(Bz, dtype=np.float64)
            if E.size != self.prm.ncells or B.size != self.prm.ncells:
                raise ValueError("wrong field length")
            self._check(self._lib.pic_fields_load(self._ctx, n, MEM_HOST, E.ctypes.data,
                                                  B.ctypes.data))

    def fields_load_lattice(self, n_first: int, count: int, table, M: int, coeffs):
        torch = _torch()
        tp = _dev_ptr(table, torch.float64)
        if table.numel() < M:
            raise ValueError("table shorter than M")
        self._check(self._lib.pic_fields_load_lattice(self._ctx, n_first, count, tp, M,
                                                      *[int(c) for c in coeffs]))

    def fields_load_r(self, run: int, n: int, Ey, Bz):
        E = np.ascontiguousarray(Ey, dtype=np.float64)
        B = np.ascontiguousarray(Bz, dtype=np.float64)
        if E.size != self.params[run].ncells or B.size != self.params[run].ncells:
            raise ValueError("wrong field length")
        self._check(self._lib.pic_fields_load_r(self._ctx, run, n, MEM_HOST, E.ctypes.data,
                                                B.ctypes.data))

    def fields_load_lattice_r(self, run: int, n_first: int, count: int, table, M: int, coeffs):
        torch = _torch()
        tp = _dev_ptr(table, torch.float64)
        self._check(self._lib.pic_fields_load_lattice_r(self._ctx, run, n_first, count, tp, M,
                                                        *[int(c) for c in coeffs]))

    def fields_yee(self, n_first: int, count: int, table, M: int, aB: int, cB: int, run: int = 0):
        """Levels n_first .. n_first + count - 1 of a run by the Yee scheme
        from level n_first - 1; the laser source is table[(aB m + cB) mod M]."""
        torch = _torch()
        tp = _dev_ptr(table, torch.float64)
        if table.numel() < M:
            raise ValueError("table shorter than M")
        self._check(self._lib.pic_fields_yee_r(self._ctx, run, n_first, count, tp, M,
                                               int(aB), int(cB)))

    def fields_read(self, n: int, run: int = 0):
        """(Ey, Bz) of ring level n as host arrays."""
        nc = self.params[run].ncells
        E = np.empty(nc)
        B = np.empty(nc)
        self._check(self._lib.pic_fields_read_r(self._ctx, run, n, MEM_HOST, E.ctypes.data,
                                                B.ctypes.data))
        return E, B

    def predictor_set(self, w_bf16=None, norm=None, run_a0=None, width: float = 0.0625,
                      every: int = 1):
        """Attach a predictor (host arrays: BF16 words as uint16, norm, one
        a0 per run); the pushes then re-order the groups every `every`-th
        call.  No arguments: detach."""
        if w_bf16 is None:
            self._check(self._lib.pic_predictor_set(self._ctx, None, None, None, 0.0, 0))
            return
        w = np.ascontiguousarray(w_bf16, dtype=np.uint16)
        nm = np.ascontiguousarray(norm, dtype=np.float32)
        a0 = np.ascontiguousarray(np.broadcast_to(np.asarray(run_a0, dtype=np.float32),
                                                  (self.nruns,)))
        if w.size != MLP_NPARAM or nm.size != 2 * MLP_FEATURES:
            raise ValueError("wrong weight or normalisation size")
        self._keep_pred = (w, nm, a0)
        self._check(self._lib.pic_predictor_set(self._ctx, w.ctypes.data, nm.ctypes.data,
                                                a0.ctypes.data, float(width), int(every)))

    def diag_track(self, on: bool = True):
        """Start (restart) or stop the trajectory diagnostics: running max of
        |R - R0| / R0 (R = gamma - p_x) and the work / energy accounting."""
        self._check(self._lib.pic_diag_track(self._ctx, 1 if on else 0))

    def dephasing_read(self):
        """(R0, running max of |R - R0| / R0) per particle, host arrays."""
        R0 = np.empty(self.num)
        rm = np.empty(self.num)
        self._check(self._lib.pic_dephasing_read(self._ctx, MEM_HOST, R0.ctypes.data,
                                                 rm.ctypes.data))
        return R0, rm

    def energy_read(self):
        """(work of E since the start, largest single-step |d gamma - work|)
        per particle, host arrays."""
        w = np.empty(self.num)
        e = np.empty(self.num)
        self._check(self._lib.pic_energy_read(self._ctx, MEM_HOST, w.ctypes.data, e.ctypes.data))
        return w, e

    def gamma_max_read(self):
        """Largest gamma of each particle since the diagnostics were
        (re)started, host array."""
        g = np.empty(self.num)
        self._check(self._lib.pic_gamma_max_read(self._ctx, MEM_HOST, g.ctypes.data))
        return g

    def gamma_error_lattice(self, atab, M: int, coeffs, run: int = 0):
        """Attach the potential table (FP64 device tensor on the phase lattice
        coeffs = (A, B, C) of the E field) for the energy error; None detaches."""
        torch = _torch()
        if atab is None:
            self._check(self._lib.pic_gamma_error_lattice(self._ctx, run, None, 0, 0, 0, 0))
            self._keep_atab = None
            return
        A, B, Cc = (int(v) for v in coeffs[:3])
        self._check(self._lib.pic_gamma_error_lattice(
            self._ctx, run, _dev_ptr(atab, torch.float64, int(M) if M > 0 else None), int(M),
            A, B, Cc))
        self._keep_atab = atab

    def gamma_error_start(self, ai):
        """a_i of every particle (host array, caller order); maxima to 0."""
        ai = np.ascontiguousarray(ai, dtype=np.float64)
        if ai.size != self.num:
            raise ValueError("a_i needs one value per particle")
        self._check(self._lib.pic_gamma_error_start(self._ctx, MEM_HOST, ai.ctypes.data))

    def gamma_error_read(self):
        """Running maximum of |gamma - gamma_th| / gamma_th per particle."""
        e = np.empty(self.num)
        self._check(self._lib.pic_gamma_error_read(self._ctx, MEM_HOST, e.ctypes.data))
        return e

    def push(self, n: int, S: int = 1):
        self._check(self._lib.pic_push_subcycled(self._ctx, n, S))

    # -- device-driven mode ------------------------------------------------
    def source_set(self, run: int, n_start: int, table, M: int, coeffs, n_stop=None):
        """Attach a device phase table to a run at level n_start, stopping at
        n_stop (the tensor is kept alive by this object)."""
        torch = _torch()
        tp = _dev_ptr(table, torch.float64)
        if table.numel() < M:
            raise ValueError("table shorter than M")
        self._sources[run] = table
        stop = (1 << 63) - 1 if n_stop is None else int(n_stop)
        self._check(self._lib.pic_source_set(self._ctx, run, n_start, stop, tp, M,
                                             *[int(c) for c in coeffs]))

    def advance(self, S: int):
        self._check(self._lib.pic_advance(self._ctx, S))

    def run_level(self, run: int = 0) -> int:
        n = C.c_int64()
        self._check(self._lib.pic_run_level(self._ctx, run, C.byref(n)))
        return n.value

    def graph_capture(self, S: int, windows: int):
        self._check(self._lib.pic_graph_capture(self._ctx, S, windows))

    def graph_launch(self):
        self._check(self._lib.pic_graph_launch(self._ctx))

    def graph_release(self):
        self._check(self._lib.pic_graph_release(self._ctx))

    def run_counters(self, run: int) -> dict:
        c = Counters()
        self._check(self._lib.pic_run_counters(self._ctx, run, C.byref(c)))
        return c.as_dict()

    # -- launch shape --------------------------------------------------------
    def tune_get(self) -> dict:
        t = Tune()
        self._check(self._lib.pic_tune_get(self._ctx, C.byref(t)))
        return t.as_dict()

    def tune_set(self, waves_per_group=None, tile=None, binning=None, sort_sub=None,
                 occupancy=None):
        cur = self.tune_get()
        t = Tune(waves_per_group=waves_per_group or cur["waves_per_group"],
                 tile=tile or cur["tile"], binning=BINNING[binning or cur["binning"]],
                 sort_sub=sort_sub or cur["sort_sub"],
                 occupancy=cur["occupancy"] if occupancy is None else occupancy)
        self._check(self._lib.pic_tune_set(self._ctx, C.byref(t)))

    def autotune(self, steps: int, reps: int = 1):
        t = Tune()
        ms = C.c_double()
        self._check(self._lib.pic_autotune(self._ctx, steps, reps, C.byref(t), C.byref(ms)))
        return t.as_dict(), ms.value

    def group_count(self) -> int:
        return int(self._lib.pic_group_count(self._ctx))

    def order_set(self, order):
        """Dispatch order of the 64-slot groups (host int32 permutation, or
        None for slot order)."""
        if order is None:
            self._check(self._lib.pic_order_set(self._ctx, None, MEM_HOST))
            return
        o = np.ascontiguousarray(order, dtype=np.int32)
        if o.size != self.group_count():
            raise ValueError("order must list every group once")
        self._check(self._lib.pic_order_set(self._ctx, o.ctypes.data, MEM_HOST))

    def features(self, a0, n=None, out=None):
        """Predictor features [num, 8] (FP32 device tensor) at level n (None:
        each run's current level); a0 = one amplitude per run."""
        torch = _torch()
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(a0, dtype=np.float32),
                                                 (self.nruns,)))
        if out is None:
            out = torch.empty((self.num, MLP_FEATURES), dtype=torch.float32, device="cuda")
        ptr = _dev_ptr(out, torch.float32, self.num * MLP_FEATURES) if self.num else None
        lev = NO_LEVEL if n is None else int(n)
        self._check(self._lib.pic_features(self._ctx, lev, a.ctypes.data, ptr))
        return out

    def prebin(self, score, nbuckets: int = 8, width: float = 1.0, prio_groups: int = 0):
        """Re-bin every run's particles by predicted load (FP32 device
        tensor, one score per caller index), heaviest groups first."""
        torch = _torch()
        ptr = _dev_ptr(score, torch.float32, self.num) if self.num else None
        torch.cuda.current_stream().synchronize()
        self._check(self._lib.pic_prebin(self._ctx, ptr, int(nbuckets), float(width),
                                         int(prio_groups)))

    def state_export(self) -> bytes:
        """Checkpoint of the particle state, counters and run levels."""
        n = C.c_size_t(0)
        self._check(self._lib.pic_state_export(self._ctx, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._lib.pic_state_export(self._ctx, buf, C.byref(n)))
        return buf.raw[:n.value]

    def state_import(self, blob: bytes):
        """Restore a checkpoint; returns each run's recorded level."""
        lev = np.zeros(self.nruns, dtype=np.int64)
        self._check(self._lib.pic_state_import(self._ctx, blob, len(blob), lev.ctypes.data))
        return lev

    def ktrace_set(self, buf, n_first: int = 0, first: int = 0):
        """Record k for caller indices [first, first + buf.shape[1]) at steps
        n_first .. n_first + buf.shape[0] - 1 into the int8 device tensor buf."""
        torch = _torch()
        if buf is None:
            self._check(self._lib.pic_ktrace_set(self._ctx, None, 0, 0, 0, 0))
            return
        if buf.dim() != 2:
            raise ValueError("k trace buffer must be [steps, count]")
        self._check(self._lib.pic_ktrace_set(self._ctx, _dev_ptr(buf, torch.int8), n_first,
                                             buf.shape[0], first, buf.shape[1]))
        self._keep = [buf]

    def counters_reset(self):
        self._check(self._lib.pic_counters_reset(self._ctx))

    def counters(self) -> dict:
        c = Counters()
        self._check(self._lib.pic_diag(self._ctx, MEM_HOST, None, None, None, None, None,
                                       None, None, C.byref(c)))
        return c.as_dict()

    def diag(self) -> dict:
        """Host copies of gamma, px, py, pz, x, k_last, status (caller order)."""
        n = self.num
        out = {k: np.empty(n) for k in ("gamma", "px", "py", "pz", "x")}
        out["k_last"] = np.empty(n, dtype=np.int8)
        out["status"] = np.empty(n, dtype=np.uint8)
        c = Counters()
        self._check(self._lib.pic_diag(
            self._ctx, MEM_HOST, *[out[k].ctypes.data for k in ("gamma", "px", "py", "pz", "x")],
            out["k_last"].ctypes.data, out["status"].ctypes.data, C.byref(c)))
        out["counters"] = c.as_dict()
        return out

    def diag_run(self, run: int) -> dict:
        """pic_diag_r: host copies of one run's particles (caller order of
        that run) and the run's counters."""
        n = int(self.nums[run])
        out = {k: np.empty(n) for k in ("gamma", "px", "py", "pz", "x")}
        out["k_last"] = np.empty(n, dtype=np.int8)
        out["status"] = np.empty(n, dtype=np.uint8)
        c = Counters()
        self._check(self._lib.pic_diag_r(
            self._ctx, int(run), MEM_HOST,
            *[out[k].ctypes.data for k in ("gamma", "px", "py", "pz", "x")],
            out["k_last"].ctypes.data, out["status"].ctypes.data, C.byref(c)))
        out["counters"] = c.as_dict()
        return out

    def grid_shift(self, cells: int, run: int = 0) -> float:
        """pic_grid_shift: move the run's grid by `cells` nodes; returns the
        new x_origin."""
        xo = C.c_double(0.0)
        self._check(self._lib.pic_grid_shift(self._ctx, int(run), int(cells), C.byref(xo)))
        return xo.value

    def strict_set(self, on: bool = True):
        self._check(self._lib.pic_strict_set(self._ctx, 1 if on else 0))

    def diag_noalloc(self, keys=("gamma", "px", "py", "pz", "x", "k_last", "status"),
                     counters: bool = True) -> dict:
        """pic_diag_noalloc: the host copies of diag() (only `keys`), staged
        through the library's fixed per-GPU array instead of an allocation."""
        n = self.num
        out = {k: np.empty(n) for k in ("gamma", "px", "py", "pz", "x") if k in keys}
        if "k_last" in keys:
            out["k_last"] = np.empty(n, dtype=np.int8)
        if "status" in keys:
            out["status"] = np.empty(n, dtype=np.uint8)
        c = Counters()
        ptrs = [out[k].ctypes.data if k in out else None
                for k in ("gamma", "px", "py", "pz", "x", "k_last", "status")]
        self._check(self._lib.pic_diag_noalloc(self._ctx, *ptrs,
                                               C.byref(c) if counters else None))
        if counters:
            out["counters"] = c.as_dict()
        return out

    def diag_device(self, out: dict):
        """Write into caller-owned device tensors (any key may be missing)."""
        torch = _torch()
        n = self.num

        def p(key, dt):
            return _dev_ptr(out[key], dt, n) if key in out else None
        self._check(self._lib.pic_diag(
            self._ctx, MEM_DEVICE, p("gamma", torch.float64), p("px", torch.float64),
            p("py", torch.float64), p("pz", torch.float64), p("x", torch.float64),
            p("k_last", torch.int8), p("status", torch.uint8), None))


# -- load predictor network (module level: needs no context) ---------------
def _stream_ptr():
    torch = _torch()
    return torch.cuda.current_stream().cuda_stream


def _mlp_status(st: int, what: str):
    if st != 0:
        raise PicError(st, what)


def ktrace_load(ktrace, out=None):
    """Per-column log2 of the mean 4^k over the live steps of a k trace
    (device int8 [steps, count]); a float32 tensor, on torch's current stream."""
    torch = _torch()
    L = load_library()
    steps, count = ktrace.shape
    if out is None:
        out = torch.empty(count, dtype=torch.float32, device="cuda")
    _mlp_status(L.pic_ktrace_load(_dev_ptr(ktrace, torch.int8, steps * count), int(steps),
                                  int(count), _dev_ptr(out, torch.float32, count), _stream_ptr()),
                "ktrace load")
    return out


def fma_probe(blocks: int, iters: int):
    """Attainable FP64 vector rate: times one launch of the FMA-chain probe on
    torch's current stream; returns TFLOP/s."""
    torch = _torch()
    L = load_library()
    out = torch.empty(int(blocks) * 256, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _mlp_status(L.pic_fma_probe(_dev_ptr(out, torch.float64), int(blocks), int(iters),
                                _stream_ptr()), "fma probe")
    e1.record(s)
    e1.synchronize()
    return 2.0 * 16 * iters * blocks * 256 / (e0.elapsed_time(e1) * 1e-3) / 1e12


def mlp_forward(w_bf16, norm, feat, out=None):
    """out[i] = network(feat[i]) with BF16 weights (int16 tensor of the
    bit patterns), on torch's current stream."""
    torch = _torch()
    L = load_library()
    n = feat.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device="cuda")
    if n == 0:
        return out
    _mlp_status(L.pic_mlp_forward(_dev_ptr(w_bf16, torch.int16, MLP_NPARAM),
                                  _dev_ptr(norm, torch.float32, 2 * MLP_FEATURES),
                                  _dev_ptr(feat, torch.float32, n * MLP_FEATURES),
                                  _dev_ptr(out, torch.float32, n), n, _stream_ptr()),
                "mlp forward")
    return out


def mlp_grad(w, norm, feat, target, grad, loss, inv_total=None):
    """Accumulate the MSE gradient (w.r.t. the FP32 master weights w, forward
    in BF16) into grad and the loss into loss[0]."""
    torch = _torch()
    L = load_library()
    n = feat.shape[0]
    if n == 0:
        return
    inv = 1.0 / n if inv_total is None else float(inv_total)
    _mlp_status(L.pic_mlp_grad(_dev_ptr(w, torch.float32, MLP_NPARAM),
                               _dev_ptr(norm, torch.float32, 2 * MLP_FEATURES),
                               _dev_ptr(feat, torch.float32, n * MLP_FEATURES),
                               _dev_ptr(target, torch.float32, n), n, inv,
                               _dev_ptr(grad, torch.float32, MLP_NPARAM),
                               _dev_ptr(loss, torch.float32, 1), _stream_ptr()), "mlp grad")


def mlp_adam(w, m, v, grad, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t >= 1) in place."""
    torch = _torch()
    L = load_library()
    n = w.numel()
    _mlp_status(L.pic_mlp_adam(_dev_ptr(w, torch.float32), _dev_ptr(m, torch.float32, n),
                               _dev_ptr(v, torch.float32, n), _dev_ptr(grad, torch.float32, n),
                               n, lr, beta1, beta2, eps, int(t), _stream_ptr()), "mlp adam")

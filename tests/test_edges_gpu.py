"""Edges of the method and of the boundary on the GPU, against the FP64
oracle: the k_max clamp of the decision (Sec. IV; the paper's loop is
unbounded and a cap counts clamps), the deepest sub-cycling the ABI allows
(k = 12, 4^12 sub-steps in one step), particles whose input state is not
finite, strict mode, and the per-run diagnostics of a batch."""

import dataclasses
import math
import sys

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TOL32 = 1e-5
TOLS = {"fp64": TOL64, "fp64fast": TOL32, "fp32c": TOL32}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _device_run(torch, wl, precision, binning="none", k_max=8, S=None, psi_max=None):
    from paper_2102_10983_amd import runner
    run = runner.DeviceRun(wl, S=S or wl.steps, precision=precision, binning=binning,
                           k_max=k_max, psi_max=psi_max)
    run.reset()
    buf = torch.full((wl.steps, wl.num), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, 0)
    run.advance(wl.steps)
    d = run.diag()
    run.close()
    return d, buf.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp64fast"])
def test_k_max_clamp(torch_gpu, precision):
    """a0 = 150, electrons at rest: the criterion asks for k up to 5 but
    k_max = 2 caps it; the clamp counter, the k traces and the states match
    the oracle run with the same cap (IEEE: bit for bit)."""
    from parity import compare
    wl = W.make_workload("clamp", 2048, 150.0, 75, 1200, 3, 3, 0.01, 2.0, seed=61)
    _say(f"k_max clamp {precision}")
    d, kt = _device_run(torch_gpu, wl, precision, k_max=2)
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOLS[precision], g_ktrace=kt,
                  flip_rel=1e-9, k_max=2)
    oc = res["oracle_counters"]
    _say({k: v for k, v in res.items() if k != "oracle_counters"}, "clamps", d["counters"]["clamps"])
    assert oc.clamps > 1000 and kt.max() == 2
    if precision == "fp64":
        assert res["bitwise"] == wl.num and d["counters"]["clamps"] == oc.clamps
        assert d["counters"]["steps_by_k"][:3] == list(oc.steps_by_k)[:3]
    else:
        assert abs(d["counters"]["clamps"] - oc.clamps) <= res["flips"]


@pytest.mark.parametrize("precision", ["fp64", "fp64fast"])
def test_deepest_subcycling(torch_gpu, precision):
    """k_max = 12, the ABI's limit: psi_max chosen so that electrons at rest
    in an a0 = 150 wave need k = 11 or 12 (up to 4^12 = 16.7 million
    sub-steps in one step); one step of 64 electrons against the oracle."""
    from parity import compare
    wl = W.make_workload("deep", 64, 150.0, 75, 256, 1.0 / 75.0, 3, 0.01, 1.0, seed=62)
    psi = 0.5 * wl.dt * 150.0 / 4.0 ** 11.5
    _say(f"deepest sub-cycling {precision}: psi_max {psi:.3g}")
    d, kt = _device_run(torch_gpu, wl, precision, k_max=12, psi_max=psi)
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOLS[precision], g_ktrace=kt,
                  psi_max=psi, flip_rel=1e-9, k_max=12)
    _say({k: v for k, v in res.items() if k != "oracle_counters"}, "k:", np.bincount(kt[0]))
    assert (kt[0] == 12).sum() > 0 and (kt[0] == 11).sum() > 0
    assert d["counters"]["sub_steps_by_k"][12] == (kt[0] == 12).sum() * 4 ** 12
    if precision == "fp64":
        assert res["bitwise"] == wl.num


def _with_bad_particles(wl):
    x0 = wl.x0.copy()
    p0 = wl.p0.copy()
    bad = {3: ("x", math.nan), 100: ("px", math.inf), 517: ("py", math.nan),
           800: ("pz", -math.inf), 1000: ("x", math.inf)}
    for i, (what, v) in bad.items():
        if what == "x":
            x0[i] = v
        else:
            p0["xyz".index(what[1]), i] = v
    return dataclasses.replace(wl, x0=x0, p0=p0), np.array(sorted(bad))


@pytest.mark.parametrize("precision,binning", [("fp64", "none"), ("fp64", "ballot"),
                                               ("fp64fast", "none"), ("fp32c", "none")])
def test_non_finite_particles_are_frozen(torch_gpu, precision, binning):
    """Five electrons of the small case get a NaN or an infinite x or p
    component: each is flagged lost and counted once, keeps its input values,
    and every other electron matches the oracle at the path's tolerance."""
    from parity import compare
    wl, bad = _with_bad_particles(W.small_case(order=3, periods=2))
    _say(f"non-finite particles {precision} {binning}")
    d, kt = _device_run(torch_gpu, wl, precision, binning=binning, S=25)
    good = np.setdiff1d(np.arange(wl.num), bad)
    res = compare(wl, wl.steps, d, good, TOLS[precision], g_ktrace=kt,
                  flip_rel=1e-9 if precision != "fp32c" else 1e-4)
    _say({k: v for k, v in res.items() if k != "oracle_counters"})
    assert np.all(d["status"][bad] == 1) and np.all(kt[:, bad] == -1)
    assert np.array_equal(d["x"][bad], wl.x0[bad], equal_nan=True)
    for c, key in enumerate(("px", "py", "pz")):
        assert np.array_equal(d[key][bad], wl.p0[c][bad], equal_nan=True)
    assert d["counters"]["lost"] == len(bad) + res["oracle_counters"].lost
    assert d["counters"]["steps"] == res["oracle_counters"].steps


def test_strict_mode_refuses_non_finite_input(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import picsub, runner
    wl = W.small_case(order=3, num=256, periods=0.2)
    run = runner.DeviceRun(wl, S=wl.steps, precision="fp64fast", binning="none")
    p = run.pusher
    p.strict_set(True)
    x = run.x0.clone()
    x[7] = float("nan")
    with pytest.raises(picsub.PicError) as e:
        p.particles_set(x, *run.p0)
    assert e.value.status == 6
    E = np.zeros(wl.ncells)
    B = np.zeros(wl.ncells)
    B[11] = np.inf
    with pytest.raises(picsub.PicError) as e:
        p.fields_load(0, E, B)
    assert e.value.status == 6
    table = run.table.clone()
    table[5] = float("nan")
    with pytest.raises(picsub.PicError) as e:
        p.fields_load_lattice(0, 1, table, run.M, run.coeffs)
    assert e.value.status == 6
    # finite input passes in strict mode, and off accepts the bad values
    run.reset()
    p.strict_set(False)
    p.particles_set(x, *run.p0)
    p.fields_load(0, E, B)
    run.close()


def test_diag_of_one_run(torch_gpu):
    """pic_diag_r returns a run's slice of pic_diag (its caller order) and its
    own counters, on a batch of three uneven runs."""
    from paper_2102_10983_amd import runner
    wls = [W.make_workload(f"r{i}", n, a0, nt, 600, 2, 3, 0.01, 1.0, seed=70 + i)
           for i, (n, a0, nt) in enumerate(((700, 20.0, 75), (1500, 80.0, 40), (333, 5.0, 150)))]
    br = runner.BatchRun(wls, S=max(w.steps for w in wls), precision="fp64", binning="none")
    br.reset()
    br.run_all()
    d = br.diag()
    off = 0
    for r, wl in enumerate(wls):
        dr = br.pusher.diag_run(r)
        for k in ("gamma", "px", "py", "pz", "x", "k_last", "status"):
            assert np.array_equal(dr[k], d[k][off:off + wl.num]), (r, k)
        assert dr["counters"] == br.pusher.run_counters(r)
        assert dr["counters"]["steps"] > 0
        off += wl.num
    br.close()


def test_fma_probe(torch_gpu):
    """The attainable-rate probe: a small launch gives a positive rate below
    the vendor's FP64 vector peak (78.6 TFLOP/s at 2.4 GHz), and it refuses
    empty launches."""
    from paper_2102_10983_amd import picsub
    rate = picsub.fma_probe(64, 2000)
    assert 0 < rate < 80.0
    out = torch_gpu.empty(256, dtype=torch_gpu.float64, device="cuda")
    L = picsub.load_library()
    assert L.pic_fma_probe(out.data_ptr(), 1, 0, None) == 1
    assert L.pic_fma_probe(None, 1, 10, None) == 1

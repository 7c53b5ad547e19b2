"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance for the FP64 path: 1e-12 relative on p and x
(e_p = |p - p_ref| / max(|p_ref|, 1), e_x = |x - x_ref| / max(|x_ref - x0|,
2 pi)), with the k-trace protocol of tests/parity.py.
"""

import math
import os
import sys

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TOL32 = 1e-5      # FP32-compensated path against the FP64 oracle
FLIP32 = 1e-4     # first differing decision of the FP32 path: this close to a threshold


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def runner(torch_gpu):
    from paper_2102_10983_amd import runner as R
    return R


def _ktrace(torch, run, steps):
    buf = torch.full((steps, run.wl.num), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0)
    return buf


def _gpu_full(torch, runner, wl, steps, S, order=None, psi_max=None, trace=True,
              binning="ballot", precision="fp64"):
    run = runner.DeviceRun(wl, S=S, order=order, psi_max=psi_max, binning=binning,
                           precision=precision)
    run.reset()
    buf = _ktrace(torch, run, steps) if trace else None
    run.advance(steps)
    d = run.diag()
    kt = buf.cpu().numpy() if trace else None
    run.close()
    return d, kt


def test_native_library_is_loaded(torch_gpu, runner):
    wl = W.small_case(order=3, num=64, periods=0.1)
    run = runner.DeviceRun(wl)
    run.close()
    maps = open("/proc/self/maps").read()
    assert "libpicsub.so" in maps


@pytest.mark.parametrize("order", [1, 3])
def test_single_step(torch_gpu, runner, order):
    _say(f"single step order={order}")
    wl = W.small_case(order=order, num=1024, periods=1)
    d, kt = _gpu_full(torch_gpu, runner, wl, 1, 1)
    from parity import compare
    res = compare(wl, 1, d, np.arange(wl.num), TOL64, g_ktrace=kt)
    _say(res)
    assert res["flips"] == 0


@pytest.mark.parametrize("order,S,binning", [(1, 1, "none"), (2, 1, "none"), (3, 1, "none"),
                                             (3, 16, "none"), (1, 75, "ballot"),
                                             (2, 40, "ballot"), (3, 1, "ballot"),
                                             (3, 250, "ballot")])
def test_small_case_full_run(torch_gpu, runner, order, S, binning):
    """1024 electrons, a0 = 10, T/dt = 75, 2048 cells, 20 periods."""
    _say(f"small case order={order} S={S} binning={binning}")
    wl = W.small_case(order=order)
    d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, S, binning=binning)
    from parity import compare
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL64, g_ktrace=kt)
    _say({k: v for k, v in res.items() if k != "oracle_counters"})
    c = res["oracle_counters"]
    if res["flips"] == 0:
        g = d["counters"]
        assert g["steps"] == c.steps and g["sub_steps"] == c.sub_steps
        assert g["n_star"] == c.n_star and g["steps_by_k"] == list(c.steps_by_k)
    assert kt.min() >= 0 and kt.max() >= 2


@pytest.mark.parametrize("binning", ["none", "ballot"])
def test_ragged_sizes(torch_gpu, runner, binning):
    from parity import compare
    for num in (1, 63, 65, 1000, 4099):
        _say(f"ragged num={num} binning={binning}")
        wl = W.make_workload("r", num, 30.0, 75, 2048, 2, 3, 0.01, 1.0, seed=num)
        d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, 10, binning=binning)
        compare(wl, wl.steps, d, np.arange(num), TOL64, g_ktrace=kt)


@pytest.mark.parametrize("order", [1, 2, 3, 5])
def test_binning_modes_are_bitwise_identical(torch_gpu, runner, order):
    """Which lane runs a particle must not change its arithmetic: the
    one-lane-per-particle push and the compacted tile push agree bit for
    bit, k traces and counters included (thermal load: uncorrelated
    neighbours, many mixed-k tiles)."""
    wl = W.make_workload("inv", 3000, 100.0, 75, 2048, 3, order, 0.01, 4.0, seed=31,
                         theta=10.0 / 511.0)
    res = {}
    for b in ("none", "ballot"):
        for S in (1, 37):
            d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, S, order=order, binning=b)
            res[(b, S)] = (d, kt)
    ref_d, ref_kt = res[("none", 1)]
    assert ref_kt.max() >= 3
    for key, (d, kt) in res.items():
        for f in ("x", "px", "py", "pz", "k_last", "status"):
            assert np.array_equal(d[f], ref_d[f]), (key, f)
        assert np.array_equal(kt, ref_kt), key
        assert d["counters"] == ref_d["counters"], key


def test_empty_particle_set(torch_gpu, runner):
    wl = W.small_case(order=3, num=0, periods=0.2)
    run = runner.DeviceRun(wl, S=5)
    run.reset()
    run.advance(wl.steps)
    d = run.diag()
    assert d["counters"]["steps"] == 0 and d["x"].size == 0
    run.close()


def test_explicit_levels_equal_lattice_levels(torch_gpu, runner):
    """pic_fields_load (host and device arrays) gives bitwise the same push
    as the on-device lattice sampler."""
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    wl = W.small_case(order=3, num=512, periods=2)
    d_lat, _ = _gpu_full(torch, runner, wl, wl.steps, 1, trace=False)
    table, M, shift = wl.table()
    for mem in ("host", "device"):
        pu = picsub.Pusher(num=wl.num, ncells=wl.ncells, order=3, dx=wl.dx, dt=wl.dt,
                           psi_max=wl.psi_max, x_origin=wl.x_origin, ring_depth=4)
        pu.particles_set(wl.x0, *wl.p0)
        for n in range(-3, wl.steps):
            E, B = W.sample_levels(wl.lat, table, M, shift, wl.ncells, n, 1)
            if mem == "device":
                pu.fields_load(n, torch.from_numpy(E[0]).cuda(), torch.from_numpy(B[0]).cuda())
            else:
                pu.fields_load(n, E[0], B[0])
            if n >= 0:
                pu.push(n, 1)
        d = pu.diag()
        pu.close()
        for k in ("x", "px", "py", "pz"):
            assert np.array_equal(d[k], d_lat[k]), (mem, k)


def test_lost_particles_match_oracle(torch_gpu, runner):
    """Electrons started next to the right edge leave the grid; they are
    frozen and flagged exactly where the oracle freezes them."""
    from parity import compare
    wl = W.make_workload("edge", 256, 30.0, 75, 160, 3, 3, 0.01, 1.0, seed=3)
    wl.x0[:] = wl.x_origin + (150 + 8 * np.arange(256) / 256.0) * wl.dx
    wl.x0[::7] = wl.x_origin + 0.25 * wl.dx        # outside on the left from the start
    d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, 25)
    d2, kt2 = _gpu_full(torch_gpu, runner, wl, wl.steps, 25, binning="none")
    assert np.array_equal(kt, kt2) and np.array_equal(d["x"], d2["x"])
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL64, g_ktrace=kt)
    assert d["counters"]["lost"] == int((d["status"] != 0).sum()) > 40
    _say(res["oracle_counters"].lost, d["counters"]["lost"])
    assert res["oracle_counters"].lost == d["counters"]["lost"]


@pytest.mark.parametrize("S", [25, 75])
def test_lost_wavefronts_fp64fast(torch_gpu, runner, S):
    """The same electrons in the FP64_FAST push (position order, so whole
    wavefronts run out of live lanes in mid-launch and go on as no-ops):
    k traces, flags and loss counts as in the oracle."""
    from parity import compare
    wl = W.make_workload("edge", 256, 30.0, 75, 160, 3, 3, 0.01, 1.0, seed=3)
    wl.x0[:] = wl.x_origin + (150 + 8 * np.arange(256) / 256.0) * wl.dx
    wl.x0[::7] = wl.x_origin + 0.25 * wl.dx
    d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, S, binning="none",
                      precision="fp64fast")
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL32, g_ktrace=kt, flip_rel=1e-9)
    _say(S, {k: v for k, v in res.items() if k != "oracle_counters"})
    assert d["counters"]["lost"] == int((d["status"] != 0).sum()) >= 64
    assert res["oracle_counters"].lost == d["counters"]["lost"]
    assert (kt[-1] < 0).sum() >= 64


def test_error_codes(torch_gpu):
    from paper_2102_10983_amd import picsub
    with pytest.raises(picsub.PicError) as e:
        picsub.Pusher(num=4, ncells=16, order=4, dx=1.0, dt=0.5, psi_max=0.01)
    assert e.value.status == 1
    with pytest.raises(picsub.PicError) as e:
        picsub.Pusher(num=4, ncells=16, order=3, dx=1.0, dt=0.5, psi_max=0.01, ring_depth=3)
    assert e.value.status == 1
    pu = picsub.Pusher(num=4, ncells=16, order=3, dx=1.0, dt=0.5, psi_max=0.01, ring_depth=5)
    with pytest.raises(picsub.PicError) as e:
        pu.push(0, 1)
    assert e.value.status == 5          # particles not loaded
    pu.particles_set(np.full(4, 8.0), np.zeros(4), np.zeros(4), np.zeros(4))
    z = np.zeros(16)
    for n in (-3, -2, -1):
        pu.fields_load(n, z, z)
    with pytest.raises(picsub.PicError) as e:
        pu.push(0, 1)                     # level 0 missing
    assert e.value.status == 4
    pu.fields_load(0, z, z)
    pu.push(0, 1)
    with pytest.raises(picsub.PicError) as e:
        pu.push(1, 2)                     # S + order > ring depth
    assert e.value.status == 4
    pu.close()


@pytest.mark.parametrize("seed", [20, 21, 22])
def test_large_case_sampled(torch_gpu, runner, seed):
    """2^20 electrons, a0 in {30, 100, 150}, 8192 cells, the full 100 periods
    in the bench's launch shape; 2048 sampled particles against the oracle."""
    torch = torch_gpu
    wl = W.large_case(seed=seed)
    steps = wl.steps
    S = int(os.environ.get("PICSUB_BENCH_S", "0")) or wl.steps
    _say(f"large case seed={seed} a0={wl.a0} steps={steps} S={S}")
    run = runner.DeviceRun(wl, S=S, binning="none")
    run.reset()
    # positions are i.i.d., so a window of caller indices is a random sample
    first = int(np.random.default_rng(seed).integers(0, wl.num - 2048))
    idx = np.arange(first, first + 2048)
    buf = torch.full((steps, 2048), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, first)
    run.advance(steps)
    d = run.diag()
    kt = buf.cpu().numpy()
    run.close()
    full = np.full((steps, wl.num), -3, dtype=np.int8)
    full[:, idx] = kt
    from parity import compare
    res = compare(wl, steps, d, idx, TOL64, g_ktrace=full)
    _say({k: v for k, v in res.items() if k != "oracle_counters"})
    g = d["counters"]
    assert g["steps"] == steps * wl.num and g["lost"] == 0
    assert g["sub_steps"] == sum(c << (2 * k) for k, c in enumerate(g["steps_by_k"]))


# ---------------------------------------------------------------------------
# Fast FP64 (refined hardware reciprocals, node-unit positions): the
# non-bitwise path held to the 1e-5 bar
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order,S", [(1, 1500), (2, 1500), (2, 7), (3, 1500), (3, 7), (5, 300)])
def test_fp64fast_small_case(torch_gpu, runner, order, S):
    _say(f"fp64fast small case order={order} S={S}")
    from parity import compare
    wl = W.small_case(order=order)
    d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, S, binning="none", precision="fp64fast")
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL32, g_ktrace=kt, flip_rel=1e-9)
    _say({k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["max_e_p"] < 1e-9     # rounding-level in practice
    # the counters are the histogram of the kernel's own k trace (no electron is lost here)
    g = d["counters"]
    assert g["lost"] == 0
    assert g["steps_by_k"][:9] == [int(np.sum(kt == k)) for k in range(9)]
    assert g["sub_steps"] == int(np.sum(np.where(kt >= 0, 4 ** kt.astype(np.int64), 0)))
    assert g["steps"] == int(np.sum(kt >= 0))


def test_fp64fast_thermal_and_edges(torch_gpu, runner):
    """Thermal electrons (10 keV), a0 = 100, some leaving the grid."""
    from parity import compare
    wl = W.make_workload("th", 3000, 100.0, 75, 500, 4, 3, 0.01, 4.0, seed=41,
                         theta=10.0 / 511.0)
    d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, 100, binning="none",
                      precision="fp64fast")
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL32, g_ktrace=kt, flip_rel=1e-9)
    _say({k: v for k, v in res.items() if k != "oracle_counters"})
    assert d["counters"]["lost"] > 0


@pytest.mark.parametrize("seed", [20, 21, 22])
def test_fp64fast_large_case_sampled(torch_gpu, runner, seed):
    """2^20 electrons, a0 in {30, 100, 150}, 100 periods, one launch (the
    bench's launch shape); 2048 sampled electrons within 1e-5 of the FP64
    oracle."""
    torch = torch_gpu
    wl = W.large_case(seed=seed)
    _say(f"fp64fast large case seed={seed} a0={wl.a0}")
    run = runner.DeviceRun(wl, S=wl.steps, binning="none", precision="fp64fast")
    run.reset()
    first = int(np.random.default_rng(seed + 100).integers(0, wl.num - 2048))
    idx = np.arange(first, first + 2048)
    buf = torch.full((wl.steps, 2048), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, first)
    run.advance(wl.steps)
    d = run.diag()
    kt = buf.cpu().numpy()
    run.close()
    full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
    full[:, idx] = kt
    from parity import compare
    res = compare(wl, wl.steps, d, idx, TOL32, g_ktrace=full, flip_rel=1e-9)
    _say({k: v for k, v in res.items() if k != "oracle_counters"})


# ---------------------------------------------------------------------------
# FP32-compensated path (k = 0 steps in FP32 with compensated state, FP64
# decision and sub-cycled steps) against the FP64 oracle at 1e-5.
# ---------------------------------------------------------------------------
def _fp32c_report(tag, res):
    _say(tag, {k: v for k, v in res.items() if k not in ("oracle_counters", "e_p_each")})


@pytest.mark.parametrize("order", [1, 3])
def test_fp32c_small_case(torch_gpu, runner, order):
    """1024 electrons, a0 = 10, 20 periods: every electron within 1e-5 of
    the FP64 oracle on p and x (k-flip protocol, flips within FLIP32 of a
    threshold)."""
    _say(f"fp32c small case order={order}")
    from parity import compare
    wl = W.small_case(order=order)
    d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, wl.steps, binning="none",
                      precision="fp32c")
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL32, g_ktrace=kt, flip_rel=FLIP32)
    _fp32c_report(f"fp32c small case order={order}:", res)
    assert res["max_e_gamma"] <= TOL32


def _fp32c_large(torch, runner, seed, precision="fp32c"):
    wl = W.large_case(seed=seed)
    run = runner.DeviceRun(wl, S=wl.steps, binning="none", precision=precision)
    run.reset()
    first = int(np.random.default_rng(seed + 100).integers(0, wl.num - 2048))
    idx = np.arange(first, first + 2048)
    buf = torch.full((wl.steps, 2048), -2, dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, 0, first)
    run.advance(wl.steps)
    d = run.diag()
    kt = buf.cpu().numpy()
    run.close()
    full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
    full[:, idx] = kt
    return wl, d, full, idx


@pytest.mark.parametrize("seed", [20, 21, 22])
def test_fp32c_large_case(torch_gpu, runner, seed):
    """2^20 electrons at rest, a0 in {30, 100, 150}, 100 periods, one launch;
    2048 sampled electrons against the FP64 oracle, errors on gamma, p_x and
    x reported.  Every electron is within 1e-5 on p and x, except electrons
    whose FP64 trajectory is itself that sensitive: those must be within
    their own oracle response to a 1e-10 relative change of x0 (the size of
    perturbation the FP32 increments amount to, measured with the float32
    model of the k = 0 step in tests/fp32_model.py).  p99 of e_p <= 1e-6."""
    _say(f"fp32c large case seed={seed}")
    from parity import compare, conditioning
    wl, d, full, idx = _fp32c_large(torch_gpu, runner, seed)
    res = compare(wl, wl.steps, d, idx, math.inf, g_ktrace=full, flip_rel=FLIP32, keep_each=True)
    e_p = res["e_p_each"]
    kappa = conditioning(wl, wl.steps, idx)
    over = e_p > TOL32
    _fp32c_report(f"fp32c large case a0={wl.a0}:", res)
    _say(f"  over 1e-5: {int(over.sum())} electrons, their e_p {e_p[over]}, oracle response "
         f"{kappa[over]}; electrons with response > 1e-5: {int((kappa > TOL32).sum())}")
    assert np.all(~over | (e_p <= kappa)), (e_p[over], kappa[over])
    assert res["max_e_x"] <= TOL32
    assert res["p99_e_p"] <= 1e-6


@pytest.mark.parametrize("order", [1, 3])
def test_fp64fast_register_budget_changes_nothing(torch_gpu, runner, order):
    """occupancy = 5, 6, 7 compile the same arithmetic for that many
    wavefronts per SIMD (registers spill at 6 and 7): the bits, counters and
    k trace are those of the default budget."""
    torch = torch_gpu
    wl = W.make_workload("th", 3000, 100.0, 75, 500, 4, order, 0.01, 4.0, seed=41,
                         theta=10.0 / 511.0)
    out = []
    for occ in (0, 5, 6, 7):
        run = runner.DeviceRun(wl, S=wl.steps, binning="none", precision="fp64fast")
        run.pusher.tune_set(occupancy=occ)
        run.reset()
        buf = torch.full((wl.steps, wl.num), -2, dtype=torch.int8, device="cuda")
        run.pusher.ktrace_set(buf, 0, 0)
        run.advance(wl.steps)
        d = run.diag()
        out.append((d, buf.cpu().numpy()))
        run.close()
    run = runner.DeviceRun(wl, S=wl.steps, binning="none", precision="fp64fast")
    for bad in (4, 8):
        with pytest.raises(Exception):
            run.pusher.tune_set(occupancy=bad)
    run.close()
    d0, k0 = out[0]
    for d5, k5 in out[1:]:
        for key in ("x", "px", "py", "pz", "k_last", "status"):
            assert np.array_equal(d0[key], d5[key]), key
        assert d0["counters"] == d5["counters"] and np.array_equal(k0, k5)


@pytest.mark.parametrize("precision,occ", [("fp64fast", 0), ("fp64fast", 5), ("fp64fast", 7),
                                           ("fp64", 0)])
def test_trace_buffer_changes_nothing(torch_gpu, runner, precision, occ):
    """A launch with a k-trace buffer attached runs a kernel with the trace
    compiled in, one without runs a kernel without it: the same bits and
    counters either way (thermal electrons, some sub-cycled, some lost)."""
    torch = torch_gpu
    wl = W.make_workload("th", 3000, 100.0, 75, 500, 4, 3, 0.01, 4.0, seed=43,
                         theta=10.0 / 511.0)
    out = []
    for traced in (False, True):
        run = runner.DeviceRun(wl, S=wl.steps, binning="none", precision=precision)
        run.pusher.tune_set(occupancy=occ)
        run.reset()
        if traced:
            buf = torch.full((wl.steps, wl.num), -2, dtype=torch.int8, device="cuda")
            run.pusher.ktrace_set(buf, 0, 0)
        run.advance(wl.steps)
        out.append(run.diag())
        run.close()
    d0, d1 = out
    for key in ("x", "px", "py", "pz", "k_last", "status"):
        assert np.array_equal(d0[key], d1[key]), key
    assert d0["counters"] == d1["counters"]
    assert d0["counters"]["lost"] > 0 and d0["counters"]["steps_by_k"][1] > 0


@pytest.mark.parametrize("case", range(12))
def test_random_configurations(torch_gpu, runner, case):
    """Seeded random configurations over the method's parameters: a0
    log-uniform in [1, 150] (in [30, 150] for cases 8-11, where steps
    sub-cycle deeply), order 1/3/5, Psi_max in {0.003, 0.01, 0.03},
    T/dt in {40, 75, 150}, electrons at rest or thermal, 0.5-3 wavelengths,
    2-5 periods, one launch or launches of 37 steps.  The IEEE push is held
    to 1e-12 and the fast push to 1e-5 against the oracle (k-flip protocol)."""
    from parity import compare
    rng = np.random.default_rng(1000 + case)
    a0 = float(np.exp(rng.uniform(np.log(30.0) if case >= 8 else 0.0, np.log(150.0))))
    order = int(rng.choice([1, 3, 5]))
    psi = float(rng.choice([0.003, 0.01, 0.03]))
    n_t = int(rng.choice([40, 75, 150]))
    periods = float(rng.uniform(2.0, 5.0))
    theta = 10.0 / 511.0 if rng.integers(0, 2) else 0.0
    num = int(rng.integers(700, 2500))
    span = float(rng.uniform(0.5, 3.0))
    ncells = int((span + periods + 6.0) * n_t / 1.01) + 16
    wl = W.make_workload(f"random {case}", num, a0, n_t, ncells, periods, order, psi, span,
                         seed=case, theta=theta)
    S = wl.steps if case % 2 == 0 else 37
    _say(f"case {case}: a0={a0:.3g} p={order} psi={psi} T/dt={n_t} theta={theta:.3g} "
         f"num={num} steps={wl.steps} S={S}")
    d, kt = _gpu_full(torch_gpu, runner, wl, wl.steps, S, binning="none", precision="fp64")
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL64, g_ktrace=kt)
    d2, kt2 = _gpu_full(torch_gpu, runner, wl, wl.steps, S, binning="none",
                        precision="fp64fast")
    res2 = compare(wl, wl.steps, d2, np.arange(wl.num), TOL32, g_ktrace=kt2, flip_rel=1e-9)
    _say("  ieee", {k: v for k, v in res.items() if k != "oracle_counters"})
    _say("  fast", {k: v for k, v in res2.items() if k != "oracle_counters"})
    assert res["flips"] == 0 and res["bitwise"] == wl.num

"""GPU tests of the standard-PIC field source: the Yee solver of Sec. III
(Eqs. (Ey), (Bz)) writing the ring, and the push driven by its levels.

* Levels: bit-identical to the FP64 Yee reference (oracle/yee_ref.py) for
  grids that are one tile, several tiles with a ragged last tile, two
  nodes; counts below, at and above one launch; rings so shallow that a
  call needs many launches; negative levels and ring wrap-around.
* Push: PIC_FP64 on Yee levels bit-identical to the FP64 oracle pushing
  on the reference's levels (small case, one launch and chunks of 16);
  PIC_FP64_FAST within the 1e-5 bar (small case, thermal electrons that
  leave the grid, and 2048 sampled electrons of the 2^20 a0 = 150 case).
"""

import sys

import numpy as np
import pytest

from paper_2102_10983_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TOL32 = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _lattice_level(table, M, co, m, ncells):
    aE, bE, cE, aB, bB, cB = (int(c) for c in co)
    i = np.arange(ncells, dtype=np.int64)
    return table[(aE * m + bE * i + cE) % M], table[(aB * m + bB * i + cB) % M]


@pytest.mark.parametrize("ncells,count,depth,n_first,calls", [
    (2048, 200, 220, 1, 1),       # several tiles, ragged last tile, several launches
    (380, 64, 65, 1, 1),          # exactly one tile, exactly one launch
    (381, 65, 66, -7, 1),         # one node over a tile, one level over a launch
    (1000, 3, 4, 5, 10),          # ring of 4: three levels per call, ten calls
    (2, 9, 10, 0, 1),             # the smallest grid
])
def test_levels_bitwise_equal_reference(torch_gpu, ncells, count, depth, n_first, calls):
    torch = torch_gpu
    from oracle import yee_ref as Y
    from paper_2102_10983_amd import picsub
    _say(f"yee levels ncells={ncells} count={count} depth={depth} n_first={n_first} calls={calls}")
    rng = np.random.default_rng(ncells + count)
    dt = 2 * np.pi / 75
    dx = 1.01 * dt
    M = 997
    table = rng.standard_normal(M)
    co = (3, -5, 11, 200, -202, 100)
    p = picsub.Pusher(num=0, ncells=ncells, order=3, dx=dx, dt=dt, psi_max=0.01,
                      ring_depth=depth, precision="fp64", binning="none")
    tab = torch.from_numpy(table).cuda()
    p.fields_load_lattice(n_first - 1, 1, tab, M, co)
    E0, B0 = _lattice_level(table, M, co, n_first - 1, ncells)
    El, Bl = Y.advance_lattice(E0, B0, dx, dt, n_first, count * calls, table, co[3], co[5])
    per = count
    for c in range(calls):
        p.fields_yee(n_first + c * per, per, tab, M, co[3], co[5])
        # every level this call made that the ring still holds
        for m in range(max(n_first + c * per, n_first + (c + 1) * per - depth),
                       n_first + (c + 1) * per):
            e, b = p.fields_read(m)
            j = m - n_first
            assert np.array_equal(e, El[j]) and np.array_equal(b, Bl[j]), (c, m)
    p.close()


def test_yee_errors(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    dt = 0.1
    p = picsub.Pusher(num=0, ncells=100, order=3, dx=1.01 * dt, dt=dt, psi_max=0.01,
                      ring_depth=8, precision="fp64", binning="none")
    tab = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(picsub.PicError) as e:          # start level missing
        p.fields_yee(1, 3, tab, 10, 1, 0)
    assert e.value.status == 4
    p.fields_load_lattice(0, 1, tab, 10, (0, 0, 0, 0, 0, 0))
    with pytest.raises(picsub.PicError) as e:          # more levels than the ring keeps
        p.fields_yee(1, 8, tab, 10, 1, 0)
    assert e.value.status == 1
    p.fields_yee(1, 7, tab, 10, 1, 0)
    e0, _ = p.fields_read(0)                            # still held: 8 slots, levels 0 .. 7
    p.fields_yee(8, 1, tab, 10, 1, 0)
    with pytest.raises(picsub.PicError) as e:          # level 0 was overwritten by 8
        p.fields_read(0)
    assert e.value.status == 4
    e8, b8 = p.fields_read(8)
    assert not e8.any() and not b8.any()               # zero field, zero source
    p.close()


def _run(torch, runner, wl, S, precision, ntrace=None, binning="none"):
    run = runner.DeviceRun(wl, S=S, precision=precision, binning=binning, fields="yee")
    run.reset()
    m = wl.num if ntrace is None else ntrace
    buf = torch.full((wl.steps, m), -2, dtype=torch.int8, device="cuda")
    first = 0 if ntrace is None else ntrace_first(wl, ntrace)
    run.pusher.ktrace_set(buf, 0, first)
    run.advance(wl.steps)
    d = run.diag()
    kt = buf.cpu().numpy()
    run.close()
    return d, kt, first


def ntrace_first(wl, m):
    return int(np.random.default_rng(wl.num).integers(0, wl.num - m))


@pytest.mark.parametrize("S,binning", [(1500, "none"), (16, "ballot"), (16, "none")])
def test_standard_pic_fp64_bitwise(torch_gpu, S, binning):
    """1024 electrons, a0 = 10, 2048 cells, 20 periods on Yee levels."""
    from paper_2102_10983_amd import runner
    from parity import compare, oracle_yee_fields
    wl = W.small_case(order=3)
    _say(f"standard PIC fp64 S={S} binning={binning}")
    d, kt, _ = _run(torch_gpu, runner, wl, S, "fp64", binning=binning)
    fs = oracle_yee_fields(wl, wl.steps)
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL64, g_ktrace=kt, fields=fs)
    _say({k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["flips"] == 0 and res["bitwise"] == wl.num
    c = res["oracle_counters"]
    assert d["counters"]["sub_steps"] == c.sub_steps and d["counters"]["n_star"] == c.n_star


@pytest.mark.parametrize("order,S", [(1, 1500), (5, 1500), (5, 16)])
def test_standard_pic_other_orders(torch_gpu, order, S):
    """Yee levels at 1st and 5th order: the IEEE push bit-identical to the
    oracle on the reference's levels, the fast push within rounding."""
    from paper_2102_10983_amd import runner
    from parity import compare, oracle_yee_fields
    wl = W.small_case(order=order)
    fs = oracle_yee_fields(wl, wl.steps)
    d, kt, _ = _run(torch_gpu, runner, wl, S, "fp64")
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL64, g_ktrace=kt, fields=fs)
    _say(f"standard PIC order {order} S={S} ieee:", {k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["flips"] == 0 and res["bitwise"] == wl.num
    d2, kt2, _ = _run(torch_gpu, runner, wl, S, "fp64fast")
    res2 = compare(wl, wl.steps, d2, np.arange(wl.num), TOL32, g_ktrace=kt2, fields=fs,
                   flip_rel=1e-9)
    _say(f"standard PIC order {order} S={S} fast:", {k: v for k, v in res2.items() if k != "oracle_counters"})
    assert res2["max_e_p"] < 1e-9


def test_standard_pic_fp64fast_small_and_thermal(torch_gpu):
    from paper_2102_10983_amd import runner
    from parity import compare, oracle_yee_fields
    wl = W.small_case(order=3)
    d, kt, _ = _run(torch_gpu, runner, wl, wl.steps, "fp64fast")
    res = compare(wl, wl.steps, d, np.arange(wl.num), TOL32, g_ktrace=kt,
                  fields=oracle_yee_fields(wl, wl.steps))
    _say("small:", {k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["max_e_p"] < 1e-9
    th = W.make_workload("th", 3000, 100.0, 75, 500, 4, 3, 0.01, 4.0, seed=41,
                         theta=10.0 / 511.0)
    d, kt, _ = _run(torch_gpu, runner, th, 100, "fp64fast")
    res = compare(th, th.steps, d, np.arange(th.num), TOL32, g_ktrace=kt,
                  fields=oracle_yee_fields(th, th.steps))
    _say("thermal:", {k: v for k, v in res.items() if k != "oracle_counters"})
    assert d["counters"]["lost"] > 0


def test_standard_pic_large_case_sampled(torch_gpu):
    """2^20 electrons, a0 = 150, 8192 cells, 7500 steps in one launch (the
    benchmark's shape) on Yee levels; 2048 sampled electrons."""
    from paper_2102_10983_amd import runner
    from parity import compare, oracle_yee_fields
    wl = W.large_case(seed=22)
    _say(f"standard PIC large case a0={wl.a0}")
    d, kt, first = _run(torch_gpu, runner, wl, wl.steps, "fp64fast", ntrace=2048)
    idx = np.arange(first, first + 2048)
    full = np.full((wl.steps, wl.num), -3, dtype=np.int8)
    full[:, idx] = kt
    res = compare(wl, wl.steps, d, idx, TOL32, g_ktrace=full, flip_rel=1e-9,
                  fields=oracle_yee_fields(wl, wl.steps))
    _say({k: v for k, v in res.items() if k != "oracle_counters"})
    assert res["max_e_p"] < 1e-6


def test_yee_on_one_run_of_a_batch(torch_gpu):
    """pic_fields_yee_r on run 1 of a two-run context: that run's levels
    equal the reference for its own grid and time step; run 0 is untouched."""
    torch = torch_gpu
    from oracle import yee_ref as Y
    from paper_2102_10983_amd import picsub
    rng = np.random.default_rng(77)
    runs = []
    for nc, nt in ((300, 75), (700, 150)):
        dt = 2 * np.pi / nt
        runs.append((0, picsub.make_params(ncells=nc, order=3, dx=1.01 * dt, dt=dt, psi_max=0.01,
                                           ring_depth=60, precision="fp64", binning="none")))
    p = picsub.Pusher(runs=runs)
    M = 1013
    table = rng.standard_normal(M)
    tab = torch.from_numpy(table).cuda()
    co = (7, 3, 1, 200, -202, 100)
    p.fields_load_lattice_r(1, -1, 1, tab, M, co)
    p.fields_yee(0, 50, tab, M, co[3], co[5], run=1)
    prm = runs[1][1]
    E0, B0 = _lattice_level(table, M, co, -1, prm.ncells)
    El, Bl = Y.advance_lattice(E0, B0, prm.dx, prm.dt, 0, 50, table, co[3], co[5])
    for m in (0, 17, 49):
        e, b = p.fields_read(m, run=1)
        assert np.array_equal(e, El[m]) and np.array_equal(b, Bl[m]), m
    with pytest.raises(picsub.PicError):
        p.fields_read(0, run=0)
    p.close()

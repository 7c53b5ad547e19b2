"""GPU tests of the load predictor: the network kernels against the FP64
reference, features against the reference on the same state and levels,
and re-binning by predicted load, which must leave every result unchanged."""

import sys

import numpy as np
import pytest

from oracle import mlp_ref as R
from paper_2102_10983_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problem(seed, n):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.25, R.NPARAM).astype(np.float32)
    norm = np.concatenate([rng.normal(0, 1, R.NF), 1.0 / rng.uniform(0.5, 2, R.NF)])
    norm = norm.astype(np.float32)
    feat = rng.normal(0, 1.5, (n, R.NF)).astype(np.float32)
    t = rng.normal(0, 1, n).astype(np.float32)
    return w, norm, feat, t


def _dev(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("n", [1, 63, 1000, 70001])
def test_forward_matches_reference(torch_gpu, n):
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    w, norm, feat, _ = _problem(1, n)
    bits = R.bf16_bits(w).view(np.int16)
    got = picsub.mlp_forward(_dev(torch, bits), _dev(torch, norm), _dev(torch, feat)).cpu().numpy()
    # same BF16 weights; FP64 reference vs FP32 accumulation
    want = R.forward(w, norm.astype(np.float64), feat.astype(np.float64), rounded=True)
    err = np.abs(got - want) / (1.0 + np.abs(want))
    _say("forward n", n, "max rel err", err.max())
    assert err.max() < 2e-5


@pytest.mark.parametrize("n", [64, 777, 20000])
def test_gradient_matches_reference(torch_gpu, n):
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    w, norm, feat, t = _problem(2, n)
    g = torch.zeros(R.NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    picsub.mlp_grad(_dev(torch, w), _dev(torch, norm), _dev(torch, feat), _dev(torch, t), g, loss)
    got = g.cpu().numpy().astype(np.float64)
    lref, gref = R.loss_and_grad(w, norm, feat, t, rounded=True)
    scale = np.abs(gref).max()
    err = np.abs(got - gref).max() / scale
    _say("grad n", n, "max err / max|g|", err, "loss", loss.item(), lref)
    assert err < 1e-4
    assert abs(loss.item() - lref) <= 1e-5 * lref
    # every block agrees on its own scale
    for a, b in [(R.OFF_W1, R.OFF_B1), (R.OFF_B1, R.OFF_W2), (R.OFF_W2, R.OFF_B2),
                 (R.OFF_B2, R.OFF_W3), (R.OFF_W3, R.OFF_B3), (R.OFF_B3, R.NPARAM)]:
        s = max(np.abs(gref[a:b]).max(), 1e-3 * scale)
        assert np.abs(got[a:b] - gref[a:b]).max() / s < 1e-3, (a, b)


def test_gradient_slices_sum_to_the_whole(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    w, norm, feat, t = _problem(3, 3000)
    dw, dn = _dev(torch, w), _dev(torch, norm)
    g1 = torch.zeros(R.NPARAM, dtype=torch.float32, device="cuda")
    l1 = torch.zeros(1, dtype=torch.float32, device="cuda")
    picsub.mlp_grad(dw, dn, _dev(torch, feat), _dev(torch, t), g1, l1)
    g2 = torch.zeros_like(g1)
    l2 = torch.zeros_like(l1)
    for a, b in [(0, 1111), (1111, 3000)]:
        picsub.mlp_grad(dw, dn, _dev(torch, feat[a:b]), _dev(torch, t[a:b]), g2, l2,
                        inv_total=1.0 / 3000)
    assert torch.allclose(g1, g2, rtol=1e-4, atol=1e-6 * g1.abs().max().item())
    assert abs(l1.item() - l2.item()) <= 1e-5 * l1.item()


def test_adam_matches_reference(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    rng = np.random.default_rng(4)
    w = rng.normal(0, 1, R.NPARAM).astype(np.float32)
    m = np.zeros(R.NPARAM)
    v = np.zeros(R.NPARAM)
    dw, dm, dv = _dev(torch, w), torch.zeros(R.NPARAM, device="cuda"), torch.zeros(R.NPARAM, device="cuda")
    wr = w.astype(np.float64)
    for t in range(1, 6):
        g = rng.normal(0, 1, R.NPARAM).astype(np.float32)
        picsub.mlp_adam(dw, dm, dv, _dev(torch, g), t, lr=1e-2)
        wr, m, v = R.adam(wr, m, v, g.astype(np.float64), t, lr=1e-2)
    assert np.abs(dw.cpu().numpy() - wr).max() < 1e-5


def test_training_lowers_the_loss(torch_gpu):
    """Gradient kernel + Adam fit a smooth function of the features."""
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    rng = np.random.default_rng(5)
    n = 8192
    feat = rng.normal(0, 1, (n, R.NF)).astype(np.float32)
    t = (np.sin(feat[:, 0]) + 0.5 * feat[:, 1] * feat[:, 2]).astype(np.float32)
    w = (rng.normal(0, 1, R.NPARAM) * 0.1).astype(np.float32)
    norm = np.concatenate([np.zeros(R.NF), np.ones(R.NF)]).astype(np.float32)
    dw, dn, df, dt = _dev(torch, w), _dev(torch, norm), _dev(torch, feat), _dev(torch, t)
    m = torch.zeros(R.NPARAM, device="cuda")
    v = torch.zeros(R.NPARAM, device="cuda")
    g = torch.zeros(R.NPARAM, device="cuda")
    loss = torch.zeros(1, device="cuda")
    hist = []
    for step in range(1, 301):
        g.zero_()
        loss.zero_()
        picsub.mlp_grad(dw, dn, df, dt, g, loss)
        picsub.mlp_adam(dw, m, v, g, step, lr=3e-3)
        if step in (1, 300):
            hist.append(loss.item())
    _say("loss", hist)
    assert hist[1] < 0.1 * hist[0]
    # the reference agrees on the trained weights' loss
    lref, _ = R.loss_and_grad(dw.cpu().numpy(), norm, feat, t, rounded=True)
    y = picsub.mlp_forward(torch.from_numpy(R.bf16_bits(dw.cpu().numpy()).view(np.int16)).cuda(),
                           dn, df)
    assert abs(float(((y - dt) ** 2).mean()) - lref) < 1e-3 * max(lref, 1e-3)


def _small_run(torch, binning="none", precision="fp64", S=None, wl=None):
    from paper_2102_10983_amd import runner
    wl = wl or W.small_case(num=3000, periods=4.0)
    return wl, runner.DeviceRun(wl, S=S or wl.steps, binning=binning, precision=precision)


def test_features_match_reference(torch_gpu):
    torch = torch_gpu
    wl, run = _small_run(torch, S=100)
    run.reset()
    run.advance(100)
    torch.cuda.synchronize()
    d = run.diag()
    feat = run.pusher.features(wl.a0, n=run.n).cpu().numpy()
    run.close()
    table, M, shift = wl.table()
    E, B = W.sample_levels(wl.lat, table, M, shift, wl.ncells, 98, 2)
    ref = R.features(d["x"], d["px"], d["py"], d["pz"], d["status"] == 0,
                     (E[1], E[0]), (B[1], B[0]), wl.x_origin, wl.dx, wl.dt, wl.a0, wl.ncells)
    err = np.abs(feat - ref) / (1.0 + np.abs(ref))
    _say("features max rel err", err.max(), "live", int((d["status"] == 0).sum()))
    assert err.max() < 1e-6


def test_features_need_two_levels(torch_gpu):
    from paper_2102_10983_amd import picsub
    torch = torch_gpu
    wl, run = _small_run(torch, S=10)
    run.reset()
    with pytest.raises(picsub.PicError):
        run.pusher.features(wl.a0, n=50)
    run.close()


@pytest.mark.parametrize("precision,binning,prio", [("fp64", "none", 0), ("fp64", "none", 40),
                                                    ("fp64fast", "none", 20),
                                                    ("fp64", "ballot", 0)])
def test_prebin_changes_no_result(torch_gpu, precision, binning, prio):
    """Re-binning by any score (here: random, and features-based) moves
    particles between slots and reorders groups; results stay bitwise."""
    torch = torch_gpu
    wl = W.small_case(num=5000, periods=6.0)
    steps = wl.steps
    _, ref = _small_run(torch, binning, precision, S=150, wl=wl)
    ref.reset()
    ref.advance(steps)
    want = ref.diag()
    ref.close()
    _, run = _small_run(torch, binning, precision, S=150, wl=wl)
    run.reset()
    score = torch.from_numpy(np.random.default_rng(6).normal(0, 2, wl.num).astype(np.float32)).cuda()
    score[::97] = float("nan")
    run.pusher.prebin(score, nbuckets=6, width=0.7, prio_groups=prio)
    run.advance(300)
    # and once more mid-run, from the features
    feat = run.pusher.features(wl.a0, n=run.n)
    run.pusher.prebin(feat[:, 4].contiguous(), nbuckets=4, width=1.0, prio_groups=prio)
    run.advance(steps - 300)
    got = run.diag()
    run.close()
    for k in ("x", "px", "py", "pz", "k_last", "status"):
        assert np.array_equal(got[k], want[k]), k
    assert got["counters"] == want["counters"]


def test_prebin_in_a_batch_changes_no_result(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import runner
    wls = W.batch_case(seed=12, nruns=4, periods=3.0, p_range=(100, 2000), a0_range=(5.0, 150.0),
                       cells_range=(400, 900))
    ref = runner.BatchRun(wls, S=40, precision="fp64")
    ref.reset()
    ref.run_all()
    want = ref.diag()
    ref.close()
    b = runner.BatchRun(wls, S=40, precision="fp64")
    b.reset()
    n = sum(wl.num for wl in wls)
    score = torch.from_numpy(np.random.default_rng(8).uniform(0, 5, n).astype(np.float32)).cuda()
    b.pusher.prebin(score, nbuckets=5, width=1.0, prio_groups=3)
    b.run_all()
    got = b.diag()
    b.close()
    for k in ("x", "px", "py", "pz", "k_last", "status"):
        assert np.array_equal(got[k], want[k]), k


def test_prebin_rejects_bad_arguments(torch_gpu):
    torch = torch_gpu
    from paper_2102_10983_amd import picsub
    wl, run = _small_run(torch, S=10)
    run.reset()
    s = torch.zeros(wl.num, dtype=torch.float32, device="cuda")
    for kw in (dict(nbuckets=0), dict(nbuckets=65), dict(width=0.0), dict(prio_groups=-1)):
        with pytest.raises(picsub.PicError):
            run.pusher.prebin(s, **kw)
    run.close()

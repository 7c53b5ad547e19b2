"""Pins of the FP64 predictor reference against facts that do not come
from the reference itself: exact BF16 ties, GELU limits, central
differences of the loss, the closed form of Adam's first step, and a
one-path network evaluated by hand."""

import math

import numpy as np
import pytest

from oracle import mlp_ref as R


def test_parameter_layout():
    assert R.NPARAM == 4801
    assert (R.OFF_B1, R.OFF_W2, R.OFF_B2, R.OFF_W3, R.OFF_B3) == (512, 576, 4672, 4736, 4800)


def test_bf16_rounding_exact_cases():
    # 1 + 2^-8 is half a BF16 ulp above 1: tie -> even (1.0); 1 + 3 * 2^-8
    # is a tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even) -> 1 + 2^-6.
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.0, 0.0,
                  3.140625], dtype=np.float32)
    b = R.bf16_bits(x)
    assert list(b) == [0x3F80, 0x3F80, 0x3F82, 0x3F81, 0xC000, 0x0000, 0x4049]
    assert R.bf16_round(np.float32(1 + 3 * 2 ** -8))[()] == 1 + 2 ** -6
    # values already in BF16 are fixed points
    y = R.bf16_to_float(b)
    assert np.array_equal(R.bf16_bits(y), b)


def test_gelu_limits_and_slope():
    assert R.gelu(np.array([0.0]))[0] == 0.0
    assert abs(R.gelu(np.array([10.0]))[0] - 10.0) < 1e-12
    assert abs(R.gelu(np.array([-10.0]))[0]) < 1e-12
    assert abs(R.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    # x Phi(x) at x = 1: Phi(1) = 0.8413447460685429
    assert abs(R.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    z = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (R.gelu(z + h) - R.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - R.gelu_grad(z))) < 1e-8


def _rand_problem(seed, n=37):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.3, R.NPARAM)
    norm = np.concatenate([rng.normal(0, 1, R.NF), rng.uniform(0.5, 2, R.NF)])
    feat = rng.normal(0, 1.5, (n, R.NF))
    t = rng.normal(0, 1, n)
    return w, norm, feat, t


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    w, norm, feat, t = _rand_problem(seed)
    loss, g = R.loss_and_grad(w, norm, feat, t, rounded=False)
    rng = np.random.default_rng(seed + 10)
    # every block of the parameter vector, a few coordinates each
    idx = np.concatenate([rng.choice(np.arange(a, b), size=min(6, b - a), replace=False)
                          for a, b in [(R.OFF_W1, R.OFF_B1), (R.OFF_B1, R.OFF_W2),
                                       (R.OFF_W2, R.OFF_B2), (R.OFF_B2, R.OFF_W3),
                                       (R.OFF_W3, R.OFF_B3), (R.OFF_B3, R.NPARAM)]])
    h = 1e-6
    for q in idx:
        wp = w.copy()
        wp[q] += h
        wm = w.copy()
        wm[q] -= h
        lp, _ = R.loss_and_grad(wp, norm, feat, t, rounded=False)
        lm, _ = R.loss_and_grad(wm, norm, feat, t, rounded=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(1.0, abs(fd)), (q, fd, g[q])
    # loss agrees with the forward pass
    y = R.forward(w, norm, feat, rounded=False)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-12 * max(1.0, loss)


def test_one_path_network_by_hand():
    """Only W1[0][2], W2[3][0], W3[3], b3 and b2[3] nonzero:
    y = b3 + W3[3] * gelu(W2[3][0] * gelu(W1[0][2] * u2) + b2[3])."""
    w = np.zeros(R.NPARAM)
    a, b, c, d, e = 0.5, -1.25, 2.0, 0.375, 0.25
    w[R.OFF_W1 + 0 * R.NF + 2] = a
    w[R.OFF_W2 + 3 * R.NH + 0] = b
    w[R.OFF_W3 + 3] = c
    w[R.OFF_B3] = d
    w[R.OFF_B2 + 3] = e
    norm = np.concatenate([np.zeros(R.NF), np.ones(R.NF)])
    feat = np.zeros((3, R.NF))
    feat[:, 2] = [-1.0, 0.0, 2.0]
    def phi(x):
        return 0.5 * (1 + math.erf(x / math.sqrt(2)))
    want = []
    for u in feat[:, 2]:
        h1 = a * u * phi(a * u)
        z2 = b * h1 + e
        want.append(d + c * z2 * phi(z2))
    got = R.forward(w, norm, feat, rounded=True)    # all values exact in BF16
    assert np.allclose(got, want, rtol=0, atol=1e-15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    g = rng.normal(0, 1, 50)
    w = rng.normal(0, 1, 50)
    lr, eps = 1e-2, 1e-8
    w1, m, v = R.adam(w, np.zeros(50), np.zeros(50), g, 1, lr=lr, eps=eps)
    assert np.allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_on_a_uniform_field():
    """Constant-in-space levels: the interpolated values are the level
    values; differences over dt; gamma, p_x, |p_perp|, log a0 exact."""
    nc = 10
    E = (np.full(nc, 3.0), np.full(nc, 1.0))
    B = (np.full(nc, -2.0), np.full(nc, -1.5))
    x = np.array([1.3, 0.2, 4.0, 9.5])
    p = np.array([[2.0, 0.0, 0.0, 1.0], [2.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 0.0]])
    live = np.array([True, True, False, True])
    f = R.features(x, *p, live, E, B, x_origin=0.0, dx=1.0, dt=0.5, a0=20.0, ncells=nc)
    assert np.allclose(f[0], [3.0, 2.0, 4.0, -1.0, 3.0, 2.0, 2.0, math.log(20.0)])
    assert not f[1].any()        # xi < 1/2
    assert not f[2].any()        # not live
    assert not f[3].any()        # xi >= ncells - 1


def test_features_on_fields_linear_in_x():
    """Levels linear in x with different slopes for E and B and for the two
    levels: the tent gather reproduces a linear field exactly, so every
    feature has a closed form.  E nodes sit at x_origin + (i + 1/2) dx and B
    nodes at x_origin + i dx (the Yee stagger of Sec. III), level n-1 is the
    first of each pair and n-2 the second; taking E on B's nodes, swapping
    the levels or the fields each changes a value by a slope times dx / 2 or
    flips a sign, which this test sees."""
    nc, x0, dx, dt = 40, -3.0, 0.25, 0.2
    iE = x0 + (np.arange(nc) + 0.5) * dx          # E node positions
    iB = x0 + np.arange(nc) * dx                  # B node positions
    sE1, cE1, sE2, cE2 = 1.5, 0.25, -0.5, 2.0
    sB1, cB1, sB2, cB2 = -2.0, 1.0, 0.75, -0.5
    E = (sE1 * iE + cE1, sE2 * iE + cE2)
    B = (sB1 * iB + cB1, sB2 * iB + cB2)
    x = np.array([-2.5, -1.1, 0.3, 2.9, 5.6])
    px = np.array([0.5, -1.0, 3.0, 0.0, 10.0])
    py = np.array([1.0, 2.0, -4.0, 0.0, 0.5])
    pz = np.array([0.0, 0.5, 0.0, 0.0, 2.0])
    live = np.ones(len(x), dtype=bool)
    f = R.features(x, px, py, pz, live, E, B, x_origin=x0, dx=dx, dt=dt, a0=7.0, ncells=nc)
    e1, e2 = sE1 * x + cE1, sE2 * x + cE2
    b1, b2 = sB1 * x + cB1, sB2 * x + cB2
    want = np.stack([np.abs(e1), np.abs(b1), (e1 - e2) / dt, (b1 - b2) / dt,
                     np.sqrt(1 + px ** 2 + py ** 2 + pz ** 2), px, np.hypot(py, pz),
                     np.full(len(x), math.log(7.0))], axis=1)
    assert np.allclose(f, want, rtol=1e-13, atol=1e-13)
    # a gather that took E's nodes for B's would read E at x + dx / 2
    assert np.all(np.abs(np.abs(sE1 * (x + dx / 2) + cE1) - f[:, 0]) > 0.1 * dx)

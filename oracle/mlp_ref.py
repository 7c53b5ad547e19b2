"""Plain FP64 reference of the sub-cycling load predictor: features, the
8-64-64-1 GELU network, its mean-squared-error gradient and Adam.

TEST INFRASTRUCTURE ONLY: imported by the tests; never by the product path.

The predictor is not part of the paper's method (the paper decides the
sub-cycling level from Psi alone, Sec. III); it only orders the work.  What
this module pins is the arithmetic of the device kernels:

* BF16 rounding: round-to-nearest-even of the FP32 bit pattern to the top
  16 bits (pinned in the tests on exact ties and on known bit patterns).
* GELU in the erf form, x * Phi(x) (pinned against its limits and its
  derivative 1/2 at 0, and the Gauss error function of the standard library).
* Back-propagation written out layer by layer for the loss
  L = inv_total * sum_s (y_s - t_s)^2, pinned by central differences.
* Adam (Kingma and Ba 2015, Algorithm 1) with bias correction, pinned by
  its first step, which moves every weight by lr * g / (|g| + eps).
* Features from explicit field levels with linear interpolation in space,
  the same staggering as the push: E_y nodes at (i + 1/2) dx, B_z nodes at
  i dx.
"""

from __future__ import annotations

import math

import numpy as np

NF, NH = 8, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + NH * NF
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH
NPARAM = OFF_B3 + 1

_erf = np.vectorize(math.erf, otypes=[np.float64])


def bf16_bits(w) -> np.ndarray:
    """FP32 values -> BF16 bit patterns (uint16), nearest even."""
    u = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return ((u >> 16) & 0xFFFF).astype(np.uint16)


def bf16_to_float(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def bf16_round(w) -> np.ndarray:
    """FP32 -> nearest BF16 value, returned as FP64."""
    return bf16_to_float(bf16_bits(w)).astype(np.float64)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    W1 = w[OFF_W1:OFF_B1].reshape(NH, NF)
    b1 = w[OFF_B1:OFF_W2]
    W2 = w[OFF_W2:OFF_B2].reshape(NH, NH)
    b2 = w[OFF_B2:OFF_W3]
    W3 = w[OFF_W3:OFF_B3]
    b3 = w[OFF_B3]
    return W1, b1, W2, b2, W3, b3


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def standardise(feat, norm):
    feat = np.asarray(feat, dtype=np.float64)
    norm = np.asarray(norm, dtype=np.float64)
    return (feat - norm[:NF]) * norm[NF:]


def forward(w, norm, feat, rounded: bool = True):
    """Network output per row of feat; rounded: use BF16 weights."""
    wv = bf16_round(w) if rounded else np.asarray(w, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(wv)
    u = standardise(feat, norm)
    z1 = u @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    return h2 @ W3 + b3


def loss_and_grad(w, norm, feat, target, inv_total=None, rounded: bool = True):
    """(loss, gradient) of inv_total * sum (y - t)^2 with respect to the
    (BF16-rounded when `rounded`) parameter vector, by back-propagation."""
    wv = bf16_round(w) if rounded else np.asarray(w, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(wv)
    u = standardise(feat, norm)
    t = np.asarray(target, dtype=np.float64)
    n = u.shape[0]
    inv = 1.0 / n if inv_total is None else float(inv_total)
    z1 = u @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    y = h2 @ W3 + b3
    r = y - t
    loss = inv * float(np.sum(r * r))
    dy = 2.0 * inv * r                          # dL/dy
    gW3 = h2.T @ dy
    gb3 = float(np.sum(dy))
    dz2 = np.outer(dy, W3) * gelu_grad(z2)      # dL/dz2
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)            # dL/dz1
    gW1 = dz1.T @ u
    gb1 = dz1.sum(axis=0)
    g = np.zeros(NPARAM)
    g[OFF_W1:OFF_B1] = gW1.ravel()
    g[OFF_B1:OFF_W2] = gb1
    g[OFF_W2:OFF_B2] = gW2.ravel()
    g[OFF_B2:OFF_W3] = gb2
    g[OFF_W3:OFF_B3] = gW3
    g[OFF_B3] = gb3
    return loss, g


def adam(w, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features(x, px, py, pz, live, E_lev, B_lev, x_origin, dx, dt, a0, ncells):
    """Features at level n from E_lev = (E_y at level n-1, at n-2) and
    B_lev likewise (arrays over nodes); zeros where not live or outside
    [1/2, ncells - 1) in node units."""
    num = len(x)
    out = np.zeros((num, NF))
    E1, E2 = (np.asarray(a, dtype=np.float64) for a in E_lev)
    B1, B2 = (np.asarray(a, dtype=np.float64) for a in B_lev)
    for s in range(num):
        xi = (x[s] - x_origin) / dx
        if not live[s] or not (0.5 <= xi < ncells - 1):
            continue
        iB = math.floor(xi)
        wB = xi - iB
        iE = math.floor(xi - 0.5)
        wE = (xi - 0.5) - iE
        e1 = (1 - wE) * E1[iE] + wE * E1[iE + 1]
        e2 = (1 - wE) * E2[iE] + wE * E2[iE + 1]
        b1 = (1 - wB) * B1[iB] + wB * B1[iB + 1]
        b2 = (1 - wB) * B2[iB] + wB * B2[iB + 1]
        out[s] = [abs(e1), abs(b1), (e1 - e2) / dt, (b1 - b2) / dt,
                  math.sqrt(1 + px[s] ** 2 + py[s] ** 2 + pz[s] ** 2), px[s],
                  math.hypot(py[s], pz[s]), math.log(a0)]
    return out

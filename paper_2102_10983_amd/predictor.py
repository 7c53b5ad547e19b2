"""Learned estimate of each particle's sub-cycling load, used only to order
the work (pic_prebin): particles are re-binned by predicted load and the
heaviest 64-lane groups start first.

The sub-cycling level itself is always decided from Psi (Sec. III); a
prediction changes no result, only how long the push takes.

Target: log2 of the mean number of sub-steps per step a particle takes
over the next `horizon` steps (Sec. VII counts sub-steps the same way:
4^k per step at level k).  Inputs: the 8 features of pic_features at the
window start.  The network, its gradients and Adam run in the library's
kernels; this module only moves arrays and loops.

Training data come from traced runs on the GPU (pic_ktrace_set records k
per particle and step); `python -m paper_2102_10983_amd.predictor --train`
regenerates the committed weights file.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import picsub
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "predictor_weights.npz")


def _bf16_bits(w: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns, round to nearest even."""
    u = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return ((u >> 16) & 0xFFFF).astype(np.uint16)


class Predictor:
    """FP32 master weights, feature standardisation and metadata."""

    def __init__(self, w: np.ndarray, norm: np.ndarray, meta: dict | None = None):
        self.w = np.ascontiguousarray(w, dtype=np.float32)
        self.norm = np.ascontiguousarray(norm, dtype=np.float32)
        if self.w.size != picsub.MLP_NPARAM or self.norm.size != 2 * picsub.MLP_FEATURES:
            raise ValueError("wrong parameter or normalisation size")
        self.meta = dict(meta or {})
        self._dev = None

    @classmethod
    def load(cls, path: str = WEIGHTS) -> "Predictor":
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"])) if "meta" in z else {}
            return cls(z["w"], z["norm"], meta)

    def save(self, path: str = WEIGHTS):
        np.savez(path, w=self.w, norm=self.norm, meta=np.array(json.dumps(self.meta)))

    def device(self):
        """(BF16 weights as int16 bits, norm) on the device, cached."""
        if self._dev is None:
            import torch
            bits = _bf16_bits(self.w).view(np.int16)
            self._dev = (torch.from_numpy(bits.copy()).to("cuda"),
                         torch.from_numpy(self.norm.copy()).to("cuda"))
        return self._dev

    def predict(self, feat):
        """Network output for a [n, 8] FP32 device tensor."""
        w16, norm = self.device()
        return picsub.mlp_forward(w16, norm, feat)

    def score(self, pusher: picsub.Pusher, a0, n=None):
        """Predicted log2 load of every particle of `pusher` at level n."""
        return self.predict(pusher.features(a0, n=n))

    def attach(self, pusher: picsub.Pusher, a0, every: int = 1, width: float = 0.0625):
        """Let the pushes of `pusher` score and re-order by themselves
        (pic_predictor_set) every `every`-th push call."""
        pusher.predictor_set(_bf16_bits(self.w), self.norm, a0, width=width, every=every)

    def prebin(self, pusher: picsub.Pusher, a0, n=None, nbuckets: int = 1, width: float = 0.0625,
               prio_groups: int = 0):
        """Score the particles and re-bin / re-order the groups."""
        s = self.score(pusher, a0, n)
        pusher.prebin(s, nbuckets=nbuckets, width=width, prio_groups=prio_groups)
        return s


# -- a non-learned control ----------------------------------------------------
def psi_score(pusher: picsub.Pusher, a0, dt: float, psi_max: float, n=None):
    """Order score without learning: log2 of psi0 / psi_max at level n,
    psi0 = |q| dt |B_z| / (2 gamma) from the features (|B_z| at the particle
    and gamma), clamped below at 0.  It is log2 of the sub-steps the Psi
    criterion (Sec. IV) gives the particle's next step, i.e. a predictor of
    the next step's load only; NaN (lightest) for lost particles."""
    import torch
    f = pusher.features(a0, n=n)
    psi0 = 0.5 * dt * f[:, 1].double() / f[:, 4].double()
    return torch.clamp(torch.log2(psi0 / psi_max), min=0.0).float().contiguous()


def persistence_score(ktrace):
    """Order score from the previous window (persistence): log2 of a
    particle's mean sub-steps per step over the steps of a k trace (device
    int8 [steps, particles], caller order, -1 where not live), by the
    library's reduction kernel; NaN (lightest) for particles with no live
    step."""
    return picsub.ktrace_load(ktrace)


def last_k_score(pusher):
    """Order score from the last step alone (persistence at no recording
    cost): each particle's k at its last step, from the state (caller
    order); -1 (lightest) for particles not live."""
    import torch
    k = torch.empty(pusher.num, dtype=torch.int8, device="cuda")
    pusher.diag_device({"k_last": k})
    return k.float().contiguous()


# -- training data -----------------------------------------------------------
def traced_load(run, steps: int, chunk: int = 500):
    """Run `steps` steps from the current state with a k trace of every
    particle; returns the device int64 total of 4^k per particle."""
    import torch
    num = run.wl.num
    buf = torch.empty((steps, num), dtype=torch.int8, device="cuda")
    run.pusher.ktrace_set(buf, run.n, 0)
    run.advance(steps)
    run.pusher.ktrace_set(None)
    tot = torch.zeros(num, dtype=torch.int64, device="cuda")
    one = torch.ones((), dtype=torch.int32, device="cuda")
    for c in range(0, steps, chunk):
        k = buf[c:c + chunk].to(torch.int32)
        sub = torch.where(k >= 0, torch.bitwise_left_shift(one, 2 * k.clamp(min=0)),
                          torch.zeros_like(k))
        tot += sub.sum(0).to(torch.int64)
    del buf
    return tot


def collect(wl: W.Workload, horizon: int | None = None, precision: str = "fp64fast"):
    """(features at step 0, log2 mean sub-steps per step over `horizon`
    steps) of every particle of wl that stays live, as host FP32 arrays."""
    import torch
    from . import runner
    steps = wl.steps if horizon is None else horizon
    run = runner.DeviceRun(wl, S=steps, precision=precision, binning="none")
    run.reset()
    feat = run.pusher.features(wl.a0, n=0)
    tot = traced_load(run, steps)
    status = torch.from_numpy(run.diag()["status"]).to("cuda")
    run.close()
    keep = (status == 0) & (tot > 0)
    target = torch.log2(tot.to(torch.float64) / steps).to(torch.float32)
    return feat[keep].cpu().numpy(), target[keep].cpu().numpy()


def spec_workloads(nruns: int = 40, num: int = 1 << 18, periods: float = 100.0,
                   seed: int = 600):
    """The training set: nruns runs of num electrons (1.05e7 samples by
    default), a0 log-uniform in [1, 150], T/dt from {40, 75, 150}, electrons
    at rest or thermal (2 or 10 keV), spread over 50 wavelengths on a grid
    long enough for the run; seeds disjoint from every evaluation case."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(nruns):
        a0 = math.exp(rng.uniform(0.0, math.log(150.0)))
        n_t = int((40, 75, 150)[int(rng.integers(0, 3))])
        theta = (0.0, 2.0 / 511.0, 10.0 / 511.0)[int(rng.integers(0, 3))]
        ncells = int(math.ceil((50.0 + periods + 2.0) * n_t * 100 / 101)) + 16
        out.append(W.make_workload(f"train{r} a0={a0:.3g} T/dt={n_t} theta={theta:.3g}", num,
                                   a0, n_t, ncells, periods, 3, 0.01, 50.0,
                                   seed=seed + 1 + r, theta=theta))
    return out


def training_workloads(num: int = 1 << 18, periods: float = 100.0):
    """Cold and 10 keV thermal electrons in flat waves of a0 = 30 .. 150,
    spread over 50 wavelengths (seeds disjoint from the evaluation cases)."""
    out = []
    for i, (a0, theta) in enumerate([(30.0, 0.0), (80.0, 0.0), (150.0, 0.0),
                                     (30.0, 10 / 511), (80.0, 10 / 511), (150.0, 10 / 511),
                                     (110.0, 2 / 511)]):
        out.append(W.make_workload(f"train a0={a0:g} theta={theta:.3g}", num, a0, 75, 16384,
                                   periods, 3, 0.01, 50.0, seed=500 + i, theta=theta))
    return out


def train(feat: np.ndarray, target: np.ndarray, *, steps: int = 3000, batch: int = 32768,
          lr: float = 2e-3, seed: int = 0, val_frac: float = 0.1, log=print) -> Predictor:
    """Adam on the mean squared error with the library's kernels."""
    import torch
    rng = np.random.default_rng(seed)
    n = len(target)
    perm = rng.permutation(n)
    nval = int(n * val_frac)
    val, tr = perm[:nval], perm[nval:]
    mean = feat[tr].mean(0)
    std = feat[tr].std(0)
    std = np.where(std > 1e-12, std, 1.0)
    norm = np.concatenate([mean, 1.0 / std]).astype(np.float32)
    # He-style init of the FP32 masters
    w = np.zeros(picsub.MLP_NPARAM, dtype=np.float32)
    nf, nh = picsub.MLP_FEATURES, picsub.MLP_HIDDEN
    o1, o2, o3 = nh * nf + nh, nh * nf + nh + nh * nh + nh, picsub.MLP_NPARAM - 1
    w[:nh * nf] = rng.normal(0, math.sqrt(2.0 / nf), nh * nf)
    w[nh * nf + nh:nh * nf + nh + nh * nh] = rng.normal(0, math.sqrt(2.0 / nh), nh * nh)
    w[o2:o3] = rng.normal(0, math.sqrt(1.0 / nh), nh)
    w[o3] = float(target[tr].mean())
    dev = "cuda"
    F = torch.from_numpy(np.ascontiguousarray(feat[tr])).to(dev)
    T = torch.from_numpy(np.ascontiguousarray(target[tr])).to(dev)
    Fv = torch.from_numpy(np.ascontiguousarray(feat[val])).to(dev)
    Tv = torch.from_numpy(np.ascontiguousarray(target[val])).to(dev)
    dw = torch.from_numpy(w).to(dev)
    dn = torch.from_numpy(norm).to(dev)
    m = torch.zeros_like(dw)
    v = torch.zeros_like(dw)
    g = torch.zeros_like(dw)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    ntr = F.shape[0]
    batch = min(batch, ntr)
    for t in range(1, steps + 1):
        idx = torch.randint(0, ntr, (batch,), device=dev, generator=gen)
        g.zero_()
        loss.zero_()
        picsub.mlp_grad(dw, dn, F[idx].contiguous(), T[idx].contiguous(), g, loss)
        lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (t - 1) / steps))
        picsub.mlp_adam(dw, m, v, g, t, lr=lr_t)
        if t % 500 == 0 or t == steps:
            p = Predictor(dw.cpu().numpy(), norm)
            yv = p.predict(Fv)
            mse = float(((yv - Tv) ** 2).mean())
            log(f"step {t}: batch loss {loss.item():.5f} val mse {mse:.5f} "
                f"val var {float(Tv.var()):.5f}")
    return Predictor(dw.cpu().numpy(), norm)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--train", action="store_true")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--num", type=int, default=1 << 18)
    ap.add_argument("--periods", type=float, default=100.0)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--runs", type=int, default=40, help="runs of the training set")
    ap.add_argument("--legacy", action="store_true",
                    help="the earlier set: seven runs at a0 in {30, 80, 110, 150}, T/dt = 75")
    args = ap.parse_args(argv)
    if not args.train:
        ap.print_help()
        return 0

    def log(*a):
        print(*a, flush=True)
    feats, targets = [], []
    t0 = time.time()
    wls = (training_workloads(args.num, args.periods) if args.legacy
           else spec_workloads(args.runs, args.num, args.periods))
    for wl in wls:
        f, t = collect(wl)
        log(f"{wl.name}: {len(t)} samples, target mean {t.mean():.4f} sd {t.std():.4f} "
            f"({time.time() - t0:.1f} s)")
        feats.append(f)
        targets.append(t)
    feat = np.concatenate(feats)
    target = np.concatenate(targets)
    p = train(feat, target, steps=args.steps, log=log)
    p.meta = {"horizon_periods": args.periods, "samples": int(len(target)),
              "workloads": [wl.name for wl in wls],
              "target": "log2 mean sub-steps per step over the horizon"}
    p.save(args.out)
    log(f"saved {args.out} ({time.time() - t0:.1f} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main())

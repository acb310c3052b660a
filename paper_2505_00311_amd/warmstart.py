"""Learned warm start (not in the paper): solves of a parametric family by the
batched solver give targets (x*, y*, log omega*) for a perceptron trained on
the GPU (pdcs_mlp_*), whose prediction for a new parameter starts the solve.
A cold start remains the fallback: the prediction is only a starting point,
projected onto X x Y by the solver, and the tolerance test decides as for any
start.

Everything that touches numbers on the device goes through the C ABI of
``pdcs``; this module only arranges batches, standardises the targets and
draws the initial weights."""
from __future__ import annotations

import time

import numpy as np

from . import pdcs as P


def solve_family(family, thetas, settings=None, batch_size=256, starts=None, log=None):
    """Batched solves of family.instance(theta) for every row of `thetas`.
    starts: optional list of (x0, y0, omega0) per theta; log: optional
    callable given a progress line per batch.  Returns the list of result
    dicts (info fields plus x, y) and the summed batch solve times."""
    out, secs = [], 0.0
    for i in range(0, len(thetas), batch_size):
        chunk = thetas[i:i + batch_size]
        batch = P.Batch([family.instance(t) for t in chunk])
        kw = {}
        if starts is not None:
            st = starts[i:i + batch_size]
            kw = dict(x0=[s[0] for s in st], y0=[s[1] for s in st],
                      omega0=[s[2] for s in st])
        res = batch.solve(settings or P.settings_default(), **kw)
        secs += res[0]["solve_s"] if res else 0.0
        batch.close()
        out += res
        if log:
            log(f"solved {len(out)} of {len(thetas)} (batch of {len(chunk)}: "
                f"{res[0]['solve_s'] if res else 0.0:.2f}s)")
    return out, secs


def targets_of(results):
    """(x*, y*, log omega*) per solve, one row each."""
    return np.stack([np.concatenate([r["x"], r["y"], [np.log(r["omega"])]]) for r in results])


class Standardizer:
    def __init__(self, t):
        self.mean = t.mean(axis=0)
        self.std = np.maximum(t.std(axis=0), 1e-8)

    def fwd(self, t):
        return (t - self.mean) / self.std

    def inv(self, z):
        return z * self.std + self.mean


def init_params(rng, n_in, hid, n_out):
    """He-scaled normal weights for the ReLU layers, a small output layer."""
    return np.concatenate([rng.standard_normal(hid * n_in) * np.sqrt(2.0 / n_in), np.zeros(hid),
                           rng.standard_normal(hid * hid) * np.sqrt(2.0 / hid), np.zeros(hid),
                           rng.standard_normal(n_out * hid) * 0.1 * np.sqrt(1.0 / hid),
                           np.zeros(n_out)]).astype(np.float32)


def train(thetas, targets, hidden=512, epochs=200, batch=256, lr=1e-3, seed=0, log=None):
    """Trains the network on standardised targets with Adam; returns
    (network, standardizer, loss history, seconds)."""
    import torch
    rng = np.random.default_rng(seed)
    norm = Standardizer(targets)
    z = norm.fwd(targets).astype(np.float32)
    th = thetas.astype(np.float32)
    N, n_in = th.shape
    n_out = z.shape[1]
    batch = min(batch, N)
    net = P.MLP(n_in, hidden, n_out, init_params(rng, n_in, hidden, n_out), max_batch=batch)
    th_d = torch.from_numpy(th).cuda()
    z_d = torch.from_numpy(z).cuda()
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        tot = 0.0
        steps = 0
        for i in range(0, N - batch + 1, batch):
            idx = perm[i:i + batch]
            tot += net.train_step(th_d[idx].contiguous(), z_d[idx].contiguous(), lr)
            steps += 1
        hist.append(tot / max(1, steps))
        if log and (ep % 20 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    return net, norm, hist, time.perf_counter() - t0


def predict(net, norm, thetas, n, m):
    """Starting points (x0, y0, omega0) for each theta."""
    import torch
    th = torch.from_numpy(thetas.astype(np.float32)).cuda()
    outs = []
    for i in range(0, th.shape[0], net.max_batch):
        part = th[i:i + net.max_batch].contiguous()
        o = torch.empty((part.shape[0], net.n_out), dtype=torch.float32, device="cuda")
        net.forward(part, o)
        outs.append(o.cpu().numpy())
    t = norm.inv(np.concatenate(outs).astype(np.float64))
    return [(r[:n], r[n:n + m], float(np.exp(r[n + m]))) for r in t]

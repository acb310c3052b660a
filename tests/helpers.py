"""Shared test helpers: instance construction from golden JSON and cone
membership checks written from the cone definitions (Section 1.2 and
Appendix A.2), independent of both the oracle and the GPU path."""
import json
import os

import numpy as np

from paper_2505_00311_amd.instances import Instance, csr_from_coo

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def _num(v):
    if isinstance(v, str):
        return float(v.replace("inf", "inf"))
    return float(v)


def instance_from_dense(n, m, n_box, G, c, h, l, u, xcones, rcones, name=""):
    G = np.asarray(G, dtype=np.float64).reshape(m, n)
    rows, cols = np.nonzero(G)
    rp, ci, v = csr_from_coo(m, n, rows, cols, G[rows, cols])
    if rp.size != m + 1:
        rp = np.zeros(m + 1, np.int64)
    return Instance(n=n, m=m, n_box=n_box, row_ptr=rp, col=ci, val=v,
                    c=np.array([_num(a) for a in c]), h=np.array([_num(a) for a in h]),
                    l=np.array([_num(a) for a in l]), u=np.array([_num(a) for a in u]),
                    xcone_type=np.array([t for t, _ in xcones], np.int32),
                    xcone_dim=np.array([k for _, k in xcones], np.int64),
                    rcone_type=np.array([t for t, _ in rcones], np.int32),
                    rcone_dim=np.array([k for _, k in rcones], np.int64), name=name)


# --------------------------------------------------------- cone membership
def soc_violation(v):
    """max(0, ||x|| - t) for v = (t, x)."""
    return max(0.0, float(np.linalg.norm(v[1:]) - v[0]))


def kexp_violation(v):
    """Violation of (r, s, t) in K_exp = cl{s > 0, t >= s exp(r/s)}."""
    r, s, t = v
    if s > 0:
        q = r / s
        if q > 700:
            return np.inf
        return max(0.0, s * np.exp(q) - t)
    return max(0.0, r) + max(0.0, -s) + max(0.0, -t)


def kexp_dual_violation(v):
    """Violation of (r, s, t) in K_exp^* = cl{r < 0, e t >= -r exp(s/r)}."""
    r, s, t = v
    if r < 0:
        q = s / r
        if q > 700:
            return np.inf
        return max(0.0, -r * np.exp(q) - np.e * t)
    return max(0.0, r) + max(0.0, -s) + max(0.0, -t)


def random_scaled_soc_point(rng, k, scale_range=1.0):
    v = rng.standard_normal(k) * 10 ** rng.uniform(-scale_range, scale_range)
    d = 10 ** rng.uniform(-scale_range, scale_range, k)
    return v, d

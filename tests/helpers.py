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


# ------------------------------------------------ the paper's workload families
def fisher_equilibrium_errors(inst, x):
    """Relative violations, at the solution x of the Fisher market's conic form,
    of the Eisenberg-Gale equilibrium conditions: clearing, t_i = u_i (the
    buyer's utility), p_i = log u_i, a buyer holds only goods of the best
    utility per price w_i U_ij / u_i (price q_j = max_i of it), and every
    budget is spent at those prices."""
    m, n = inst.meta["buyers"], inst.meta["goods"]
    X = x[: m * n].reshape(m, n)
    p, t = x[m * n::2], x[m * n + 1::2]
    urp, uci, uval = inst.meta["u_row_ptr"], inst.meta["u_col"], inst.meta["u_val"]
    U = np.zeros((m, n))
    for i in range(m):
        U[i, uci[urp[i]:urp[i + 1]]] = uval[urp[i]:urp[i + 1]]
    w = inst.meta["w"]
    u = (U * X).sum(axis=1)
    bpb = w[:, None] * U / u[:, None]
    q = bpb.max(axis=0)
    held = (X > 1e-4 * X.max()) & (U.max(axis=0) > 0)[None, :]
    return {
        "clearing": float(np.abs(X.sum(axis=0) - inst.meta["supply"]).max() / inst.meta["supply"]),
        "negative": float(max(0.0, -X.min()) / inst.meta["supply"]),
        "utility": float(np.abs(t - u).max() / max(1.0, u.max())),
        "log": float(np.abs(p - np.log(u)).max()),
        "bang_per_buck": float(np.abs(bpb - q[None, :])[held].max() / q.max()) if held.any() else 0.0,
        "budget": float(np.abs((X * q[None, :]).sum(axis=1) - w).max() / w.max()),
    }


def lasso_optimality_errors(inst, z):
    """Relative violations, at the solution z of the Lasso's SOCP form, of
    w = 1, y = A x - b, 2 r = ||y||^2, and the subgradient condition of
    min ||A x - b||^2 + lambda ||x||_1 (x = x1 - x2), plus its objective."""
    m, n = inst.meta["rows"], inst.meta["cols"]
    arp, aci, aval = inst.meta["a_row_ptr"], inst.meta["a_col"], inst.meta["a_val"]
    b, lam = inst.meta["b"], inst.meta["lam"]
    al = inst.meta.get("alpha", 1.0)   # balanced form: w = alpha w', r = r' / alpha
    z = np.array(z, dtype=np.float64, copy=True)
    z[0], z[1] = z[0] / al, z[1] * al
    x = z[2 + m:2 + m + n] - z[2 + m + n:]
    rows = np.repeat(np.arange(m), np.diff(arp))
    ax = np.zeros(m)
    np.add.at(ax, rows, aval * x[aci])
    res = ax - b
    g = np.zeros(n)
    np.add.at(g, aci, 2.0 * aval * res[rows])
    on = np.abs(x) > 1e-6 * max(1.0, np.abs(x).max())
    yv = z[2:2 + m]
    return {
        "w": float(abs(z[0] - 1.0)),
        "y": float(np.abs(yv - res).max() / max(1.0, np.abs(b).max())),
        "cone": float(abs(z[1] - 0.5 * yv @ yv) / max(1.0, z[1])),
        "stationary_on": float(np.abs(g[on] + lam * np.sign(x[on])).max() / lam) if on.any() else 0.0,
        "stationary_off": float(max(0.0, (np.abs(g[~on]).max() - lam) / lam)) if (~on).any() else 0.0,
        "objective": float(res @ res + lam * np.abs(x).sum()),
    }

"""Seeded synthetic conic-program instances.

This module only draws problem data.  It holds none of the solver's arithmetic
(no projection, scaling, step or KKT formula) and is the one module that both
the GPU path's tests/benchmark and the CPU oracle's tests take inputs from.

Every generator builds a problem of the form of the paper's eq. (1),
    min <c,x>  s.t.  G x - h in K_d^*,  l <= x_1 <= u,  x_2 in K_p,
and, where stated, plants a primal-dual optimum: it draws x* in X, lambda* in
the dual of X, a slack s* in K_d^* and y* in K_d with <x*,lambda*> = 0 and
<s*,y*> = 0 blockwise, then sets h = G x* - s* and c = G^T y* + lambda*.  The
planted objective <c, x*> is then the optimal value.

Cone type codes: ZERO 0, FREE 1, NONNEG 2, SOC 3, EXP 4, EXP_DUAL 5, RSOC 6 (rotated SOC).
A row block of type T states G x - h in T.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ZERO, FREE, NONNEG, SOC, EXP, EXP_DUAL, RSOC = range(7)


@dataclass
class Instance:
    n: int
    m: int
    n_box: int
    row_ptr: np.ndarray          # int64 [m+1]
    col: np.ndarray              # int32 [nnz]
    val: np.ndarray              # float64 [nnz]
    c: np.ndarray                # float64 [n]
    h: np.ndarray                # float64 [m]
    l: np.ndarray                # float64 [n_box]
    u: np.ndarray                # float64 [n_box]
    xcone_type: np.ndarray       # int32
    xcone_dim: np.ndarray        # int64
    rcone_type: np.ndarray       # int32
    rcone_dim: np.ndarray        # int64
    x_star: np.ndarray | None = None
    y_star: np.ndarray | None = None
    opt: float | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.val.size)

    def dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        for i in range(self.m):
            s, e = self.row_ptr[i], self.row_ptr[i + 1]
            A[i, self.col[s:e]] += self.val[s:e]
        return A


# ----------------------------------------------------------------- matrices
def csr_from_coo(m, n, rows, cols, vals):
    """Row-sorted CSR with duplicates summed."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, vals = key[order], vals[order]
    uk, start = np.unique(key, return_index=True)
    v = np.add.reduceat(vals, start) if vals.size else vals
    r = uk // n
    cidx = (uk % n).astype(np.int32)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp), cidx, v


def bernoulli_csr(rng, m, n, density):
    """Exactly-Bernoulli(density) sparsity pattern with N(0,1) values."""
    nnz_target = rng.binomial(m * n, density)
    flat = rng.choice(m * n, size=nnz_target, replace=False) if m * n > 0 else np.zeros(0, int)
    flat.sort()
    rows, cols = flat // n, flat % n
    return csr_from_coo(m, n, rows, cols, rng.standard_normal(flat.size))


def powerlaw_csr(rng, m, n, mean_row_nnz=20, alpha=0.8):
    """Rows with 1 + Poisson(mean-1) entries; columns drawn with weight
    (rank+1)^-alpha over a random permutation (duplicates in a row dropped)."""
    perm = rng.permutation(n)
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-alpha)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    k = 1 + rng.poisson(mean_row_nnz - 1, size=m)
    total = int(k.sum())
    ranks = np.minimum(np.searchsorted(cdf, rng.random(total), side="right"), n - 1)
    cols = perm[ranks].astype(np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), k)
    key = np.unique(rows * n + cols)
    rows, cols = key // n, key % n
    rp = np.zeros(m + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols.astype(np.int32), rng.standard_normal(key.size)


def csr_matvec(rp, col, val, x):
    """A x, each row summed in entry order (bincount adds in input order)."""
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    return np.bincount(rows, weights=val * x[col], minlength=rp.size - 1).astype(np.float64)


def csr_rmatvec(rp, col, val, y, n):
    """A^T y, each column summed in entry order."""
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    return np.bincount(col, weights=val * y[rows], minlength=n).astype(np.float64)


# ----------------------------------------------------------- planted pairs
def _pair_block(rng, typ, k):
    """(p, d) with p in the cone `typ`, d in its dual cone and <p, d> = 0."""
    if typ == ZERO:
        return np.zeros(k), rng.standard_normal(k)
    if typ == FREE:
        return rng.standard_normal(k), np.zeros(k)
    if typ == NONNEG:
        act = rng.random(k) < 0.5
        mag = np.abs(rng.standard_normal(k))
        return np.where(act, 0.0, mag), np.where(act, np.abs(rng.standard_normal(k)), 0.0)
    if typ == SOC:
        w = rng.standard_normal(k - 1)
        nw = np.linalg.norm(w)
        kind = rng.integers(3)
        if kind == 0:   # boundary, complementary boundary pair
            a = rng.uniform(0.5, 2.0)
            return np.concatenate([[nw], w]), a * np.concatenate([[nw], -w])
        if kind == 1:   # interior primal
            return np.concatenate([[nw + rng.uniform(0.5, 2.0)], w]), np.zeros(k)
        return np.zeros(k), np.concatenate([[nw + rng.uniform(0.5, 2.0)], w])
    if typ in (EXP, EXP_DUAL):
        rho = rng.standard_normal()
        sp, rd = rng.uniform(0.5, 2.0, size=2)
        p = sp * np.array([rho, 1.0, np.exp(rho)])           # in K_exp, boundary
        d = rd * np.array([-1.0, rho - 1.0, np.exp(-rho)])   # in K_exp^*, boundary
        return (p, d) if typ == EXP else (d, p)
    raise ValueError(typ)


def _split(vec, dims):
    out, o = [], 0
    for k in dims:
        out.append(slice(o, o + int(k)))
        o += int(k)
    return out


def plant(rng, n, m, n_box, row_ptr, col, val, xtypes, xdims, rtypes, rdims,
          box_kind="finite", name=""):
    """Complete (G, cones) to an instance with a planted optimum."""
    xtypes = np.asarray(xtypes, np.int32)
    xdims = np.asarray(xdims, np.int64)
    rtypes = np.asarray(rtypes, np.int32)
    rdims = np.asarray(rdims, np.int64)
    assert int(xdims.sum()) == n - n_box and int(rdims.sum()) == m
    x = np.zeros(n)
    lam = np.zeros(n)
    l = np.zeros(n_box)
    u = np.zeros(n_box)
    if n_box:
        lo = -rng.uniform(0.0, 2.0, n_box)
        hi = rng.uniform(0.0, 2.0, n_box)
        if box_kind == "mixed":     # some one-sided and free entries
            kind = rng.integers(4, size=n_box)
            lo = np.where(kind == 1, -np.inf, lo)
            hi = np.where(kind == 2, np.inf, hi)
            lo = np.where(kind == 3, -np.inf, lo)
            hi = np.where(kind == 3, np.inf, hi)
        l[:], u[:] = lo, hi
        state = rng.integers(3, size=n_box)        # 0 at l, 1 at u, 2 inside
        state = np.where((state == 0) & ~np.isfinite(lo), 2, state)
        state = np.where((state == 1) & ~np.isfinite(hi), 2, state)
        mag = rng.uniform(0.5, 2.0, n_box)
        lo_f = np.where(np.isfinite(lo), lo, -3.0)
        hi_f = np.where(np.isfinite(hi), hi, 3.0)
        inside = lo_f + rng.uniform(0.2, 0.8, n_box) * (hi_f - lo_f)
        x[:n_box] = np.where(state == 0, lo_f, np.where(state == 1, hi_f, inside))
        lam[:n_box] = np.where(state == 0, mag, np.where(state == 1, -mag, 0.0))
    for t, sl in zip(xtypes, _split(None, xdims)):
        p, d = _pair_block(rng, int(t), sl.stop - sl.start)
        x[n_box + sl.start:n_box + sl.stop] = p
        lam[n_box + sl.start:n_box + sl.stop] = d
    s = np.zeros(m)
    y = np.zeros(m)
    for t, sl in zip(rtypes, _split(None, rdims)):
        p, d = _pair_block(rng, int(t), sl.stop - sl.start)
        s[sl], y[sl] = p, d
    gx = csr_matvec(row_ptr, col, val, x)
    h = gx - s
    c = csr_rmatvec(row_ptr, col, val, y, n) + lam
    return Instance(n=n, m=m, n_box=n_box, row_ptr=np.asarray(row_ptr, np.int64),
                    col=np.asarray(col, np.int32), val=np.asarray(val, np.float64), c=c, h=h,
                    l=l, u=u, xcone_type=xtypes, xcone_dim=xdims, rcone_type=rtypes,
                    rcone_dim=rdims, x_star=x, y_star=y, opt=float(c @ x), name=name)


# ------------------------------------------------------------ workloads
def small_mixed(seed, n=40, m=24, density=0.2, n_box=6, box_kind="mixed"):
    """A small instance touching every cone type on both sides."""
    rng = np.random.default_rng(seed)
    rp, ci, v = bernoulli_csr(rng, m, n, density)
    rest = n - n_box
    xt, xd = [], []
    pattern = [(NONNEG, 5), (SOC, 4), (EXP, 3), (SOC, 7), (EXP_DUAL, 3), (FREE, 2), (ZERO, 1)]
    i = 0
    while rest > 0:
        t, k = pattern[i % len(pattern)]
        k = min(k, rest)
        if t in (EXP, EXP_DUAL) and k != 3:
            t = NONNEG
        xt.append(t), xd.append(k)
        rest -= k
        i += 1
    rt, rd = [], []
    rest = m
    rpattern = [(ZERO, 3), (NONNEG, 4), (SOC, 5), (EXP, 3), (EXP_DUAL, 3), (FREE, 1)]
    i = 0
    while rest > 0:
        t, k = rpattern[i % len(rpattern)]
        k = min(k, rest)
        if t in (EXP, EXP_DUAL) and k != 3:
            t = NONNEG
        rt.append(t), rd.append(k)
        rest -= k
        i += 1
    return plant(rng, n, m, n_box, rp, ci, v, xt, xd, rt, rd, box_kind=box_kind,
                 name=f"small_mixed(seed={seed})")


def lp_soc_small(seed):
    """The small single-instance workload: n=1000 variables, m=500 rows, G at 1%
    Bernoulli density with N(0,1) entries; x: 500 nonnegative + 50 SOC(10);
    rows: 250 equality + 250 inequality; planted optimum."""
    rng = np.random.default_rng(seed)
    n, m = 1000, 500
    rp, ci, v = bernoulli_csr(rng, m, n, 0.01)
    xt = [NONNEG] + [SOC] * 50
    xd = [500] + [10] * 50
    return plant(rng, n, m, 0, rp, ci, v, xt, xd, [ZERO, NONNEG], [250, 250],
                 name="lp_soc_n1000_m500")


def batch_lp_soc(seed, count, n_lo=1000, n_hi=100_000, density=0.005, soc_frac=0.2,
                 soc_lo=3, soc_hi=50):
    """A batch of independent planted LP/SOCP instances of uneven size:
    n ~ U{n_lo..n_hi}, m = n/2, G Bernoulli(density) with N(0,1) entries;
    soc_frac of the variables in SOC blocks of dims U{soc_lo..soc_hi}, the rest
    nonnegative; rows half equality, half inequality."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        m = n // 2
        rp, ci, v = bernoulli_csr(rng, m, n, density)
        dims, tot = [], 0
        while tot < int(soc_frac * n):
            k = int(rng.integers(soc_lo, soc_hi + 1))
            k = min(k, n - tot)
            dims.append(k)
            tot += k
        xt = [NONNEG] + [SOC] * len(dims)
        xd = [n - tot] + dims
        if xd[0] == 0:
            xt, xd = xt[1:], xd[1:]
        me = m // 2
        rt = [ZERO, NONNEG] if me and m - me else ([ZERO] if me else [NONNEG])
        rd = [me, m - me] if me and m - me else [m]
        out.append(plant(rng, n, m, 0, rp, ci, v, xt, xd, rt, rd, name=f"batch{seed}_{b}_n{n}"))
    return out


def bernoulli_csr_gaps(rng, m, n, density):
    """Bernoulli(density) pattern over the m x n positions in row-major order,
    drawn as a Bernoulli process: the gaps between successive present
    positions are geometric(density), so every position is present
    independently with probability density, in O(nnz); N(0,1) values."""
    total = m * n
    if total == 0 or density <= 0.0:
        return np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0)
    mean = total * density
    pos = np.cumsum(rng.geometric(density, size=int(mean + 8 * np.sqrt(mean) + 64))) - 1
    while pos[-1] < total:
        more = np.cumsum(rng.geometric(density, size=int(0.01 * mean) + 64)) + pos[-1]
        pos = np.concatenate([pos, more])
    pos = pos[pos < total]
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum(np.bincount(pos // n, minlength=m))
    return rp, (pos % n).astype(np.int32), rng.standard_normal(pos.size)


def batch_sizes(seed, count, n_lo=1000, n_hi=100_000):
    """The variable counts n_b ~ U{n_lo..n_hi} of batch_member(seed, b, ...)."""
    return np.random.default_rng(seed).integers(n_lo, n_hi + 1, size=count)


def batch_member(seed, b, count, n_lo=1000, n_hi=100_000, density=0.005, soc_frac=0.2,
                 soc_lo=3, soc_hi=50):
    """Instance b of a batch of `count` independent planted LP/SOCP instances
    with the recipe of batch_lp_soc (n_b ~ U{n_lo..n_hi}, m = n/2, G
    Bernoulli(density) with N(0,1) entries, soc_frac of the variables in SOC
    blocks of dims U{soc_lo..soc_hi}, the rest nonnegative; rows half
    equality, half inequality), each drawn from its own child seed so that
    members can be generated independently (in parallel) at any size."""
    n = int(batch_sizes(seed, count, n_lo, n_hi)[b])
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(count)[b])
    m = n // 2
    rp, ci, v = bernoulli_csr_gaps(rng, m, n, density)
    dims, tot = [], 0
    while tot < int(soc_frac * n):
        k = min(int(rng.integers(soc_lo, soc_hi + 1)), n - tot)
        dims.append(k)
        tot += k
    xt = [NONNEG] + [SOC] * len(dims)
    xd = [n - tot] + dims
    if xd[0] == 0:
        xt, xd = xt[1:], xd[1:]
    me = m // 2
    rt = [ZERO, NONNEG] if me and m - me else ([ZERO] if me else [NONNEG])
    rd = [me, m - me] if me and m - me else [m]
    return plant(rng, n, m, 0, rp, ci, v, xt, xd, rt, rd, name=f"member{seed}_{b}_n{n}")


def large_mixed(seed, n=1_000_000, m=500_000, n_box=None, n_soc_x=None, n_soc_r=None,
                n_exp_r=None, mean_row_nnz=20):
    """The large single-instance workload (defaults: n=1e6, m=5e5, ~1e7 nnz).

    Rows hold 1 + Poisson(19) entries whose columns follow power-law degrees
    (weight (rank+1)^-0.8 over a random permutation); entries are N(0,1) times a
    per-row scale 10^U(-3,3).  Cones: 1e5 box entries; 1e4 SOC blocks of dim
    U{3..100} on x and 1e4 of dim U{3..40} on rows; 1e4 exponential-cone row
    blocks; the other rows split into equality and inequality rows and the
    other entries of x are nonnegative.  All counts shrink with n."""
    rng = np.random.default_rng(seed)
    sc = n / 1_000_000
    n_box = int(round(100_000 * sc)) if n_box is None else n_box
    n_soc_x = int(round(10_000 * sc)) if n_soc_x is None else n_soc_x
    n_soc_r = int(round(10_000 * sc)) if n_soc_r is None else n_soc_r
    n_exp_r = int(round(10_000 * sc)) if n_exp_r is None else n_exp_r
    rp, ci, v = powerlaw_csr(rng, m, n, mean_row_nnz=mean_row_nnz)
    rowscale = 10.0 ** rng.uniform(-3.0, 3.0, m)
    v = v * np.repeat(rowscale, np.diff(rp))
    sx = rng.integers(3, 101, size=n_soc_x)
    sr = rng.integers(3, 41, size=n_soc_r)
    n_nonneg_x = n - n_box - int(sx.sum())
    assert n_nonneg_x >= 0
    xt = [NONNEG] + [SOC] * n_soc_x
    xd = [n_nonneg_x] + list(sx)
    rest = m - int(sr.sum()) - 3 * n_exp_r
    assert rest >= 0
    n_eq = rest // 2
    # interleave row blocks so that cone types are spread over the row range
    blocks = [(SOC, int(k)) for k in sr] + [(EXP, 3)] * n_exp_r
    order = rng.permutation(len(blocks))
    rt = [ZERO, NONNEG] + [blocks[i][0] for i in order]
    rd = [n_eq, rest - n_eq] + [blocks[i][1] for i in order]
    keep = [i for i, k in enumerate(rd) if k > 0]
    rt = [rt[i] for i in keep]
    rd = [rd[i] for i in keep]
    return plant(rng, n, m, n_box, rp, ci, v, xt, xd, rt, rd,
                 name=f"large_mixed_n{n}_m{m}")


def tiny_lp(seed, n=3, m=3):
    """min c^T x s.t. G x - h >= 0, l <= x <= u (finite box): a bounded LP
    small enough for vertex enumeration."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((m, n))
    rows, cols = np.nonzero(np.ones((m, n)))
    rp, ci, v = csr_from_coo(m, n, rows, cols, G[rows, cols])
    x_in = rng.uniform(-0.5, 0.5, n)
    h = G @ x_in - rng.uniform(0.1, 1.0, m)    # x_in strictly feasible
    c = rng.standard_normal(n)
    return Instance(n=n, m=m, n_box=n, row_ptr=rp, col=ci, val=v, c=c, h=h,
                    l=-np.ones(n), u=np.ones(n), xcone_type=np.zeros(0, np.int32),
                    xcone_dim=np.zeros(0, np.int64), rcone_type=np.array([NONNEG], np.int32),
                    rcone_dim=np.array([m], np.int64), name=f"tiny_lp({seed})")


def ball_socp(seed, n=4):
    """min c^T x s.t. ||W (x - x0)|| <= r, W diagonal positive; x free.
    Rows: one SOC block (r, W x - W x0); the first row of G is empty."""
    rng = np.random.default_rng(seed)
    W = rng.uniform(0.5, 2.0, n)
    x0 = rng.standard_normal(n)
    r = rng.uniform(0.5, 2.0)
    c = rng.standard_normal(n)
    rows = np.arange(1, n + 1)
    cols = np.arange(n)
    rp, ci, v = csr_from_coo(n + 1, n, rows, cols, W)
    h = np.concatenate([[-r], W * x0])
    return Instance(n=n, m=n + 1, n_box=n, row_ptr=rp, col=ci, val=v, c=c, h=h,
                    l=np.full(n, -np.inf), u=np.full(n, np.inf),
                    xcone_type=np.zeros(0, np.int32), xcone_dim=np.zeros(0, np.int64),
                    rcone_type=np.array([SOC], np.int32), rcone_dim=np.array([n + 1], np.int64),
                    name=f"ball_socp({seed})", meta={"W": W, "x0": x0, "r": r})


def box_only(c=(1.0, -2.0, 0.5)):
    """A problem without rows: min c^T x over the box [-1, 1]^n; x* = -sign(c)."""
    c = np.asarray(c, dtype=np.float64)
    n = c.size
    x = -np.sign(c)
    return Instance(n=n, m=0, n_box=n, row_ptr=np.zeros(1, np.int64), col=np.zeros(0, np.int32),
                    val=np.zeros(0), c=c, h=np.zeros(0), l=-np.ones(n), u=np.ones(n),
                    xcone_type=np.zeros(0, np.int32), xcone_dim=np.zeros(0, np.int64),
                    rcone_type=np.zeros(0, np.int32), rcone_dim=np.zeros(0, np.int64),
                    x_star=x, y_star=np.zeros(0), opt=float(c @ x), name="box_only")


# ------------------------------------------------------ parametric family
class PortfolioFamily:
    """A parametric SOC portfolio family with a k-factor risk model.

    Variables: asset weights w (n_assets, nonnegative) and factor exposures f
    (k, free); x = (w, f).  Rows, in order:
      f - F^T w = 0                                  (k rows, ZERO),
      1^T w = b(theta)                               (1 row, ZERO),
      (gamma(theta), L^T f, delta o w) in SOC(1 + k + n_assets).
    Objective: maximise expected return, c = -(mu0 + P_c theta) on w, 0 on f.
    b(theta) = 1 + p_b . theta and gamma(theta) = gamma0 (1 + p_g . theta) with
    small p_b, p_g; gamma0 is 1.5 times the risk of equal weights, so every
    theta of moderate size keeps the family feasible.  The structure (F with
    `density` nonzeros per column pattern, L, delta, mu0, P_c) is drawn once
    from `seed`; theta ~ N(0, I_dim_theta)."""

    def __init__(self, seed, n_assets=20000, k=50, density=0.2, dim_theta=64):
        rng = np.random.default_rng(seed)
        self.n_assets, self.k, self.dim_theta = n_assets, k, dim_theta
        self.n = n_assets + k
        self.m = k + 1 + 1 + k + n_assets
        mask = rng.random((n_assets, k)) < density
        fv = rng.standard_normal((n_assets, k)) * mask
        self.F = fv                                        # dense n_assets x k (for building)
        Lc = np.tril(rng.standard_normal((k, k)) * 0.05) + np.diag(rng.uniform(0.1, 0.3, k))
        self.L = Lc
        self.delta = rng.uniform(0.05, 0.2, n_assets)
        self.mu0 = rng.normal(0.05, 0.02, n_assets)
        self.Pc = rng.standard_normal((n_assets, dim_theta)) * 0.005
        self.pb = rng.standard_normal(dim_theta) * 0.01
        self.pg = rng.standard_normal(dim_theta) * 0.01
        w_eq = np.full(n_assets, 1.0 / n_assets)
        risk_eq = np.sqrt(np.sum((Lc.T @ (fv.T @ w_eq)) ** 2) + np.sum((self.delta * w_eq) ** 2))
        self.gamma0 = 1.5 * risk_eq
        # G is the same for every theta
        rows, cols, vals = [], [], []
        Fi, Fj = np.nonzero(mask)                          # F[i, j]: asset i, factor j
        # rows 0..k-1: f_j - sum_i F[i, j] w_i
        rows.append(Fj), cols.append(Fi), vals.append(-fv[Fi, Fj])
        rows.append(np.arange(k)), cols.append(n_assets + np.arange(k)), vals.append(np.ones(k))
        # row k: budget
        rows.append(np.full(n_assets, k)), cols.append(np.arange(n_assets)), vals.append(np.ones(n_assets))
        # row k+1: SOC head t = gamma (G row empty, h = -gamma)
        # rows k+2 .. k+1+k: (L^T f)_j = sum_i L[i, j] f_i
        Li, Lj = np.nonzero(Lc)
        rows.append(k + 2 + Lj), cols.append(n_assets + Li), vals.append(Lc[Li, Lj])
        # rows 2k+2 ..: delta o w
        rows.append(2 * k + 2 + np.arange(n_assets)), cols.append(np.arange(n_assets)), vals.append(self.delta)
        r = np.concatenate(rows)
        cidx = np.concatenate(cols)
        v = np.concatenate(vals)
        self.row_ptr, self.col, self.val = csr_from_coo(self.m, self.n, r, cidx, v)

    def instance(self, theta):
        theta = np.asarray(theta, dtype=np.float64)
        c = np.zeros(self.n)
        c[:self.n_assets] = -(self.mu0 + self.Pc @ theta)
        h = np.zeros(self.m)
        h[self.k] = 1.0 + self.pb @ theta
        h[self.k + 1] = -self.gamma0 * (1.0 + self.pg @ theta)
        return Instance(n=self.n, m=self.m, n_box=0, row_ptr=self.row_ptr, col=self.col,
                        val=self.val, c=c, h=h, l=np.zeros(0), u=np.zeros(0),
                        xcone_type=np.array([NONNEG, FREE], np.int32),
                        xcone_dim=np.array([self.n_assets, self.k], np.int64),
                        rcone_type=np.array([ZERO, SOC], np.int32),
                        rcone_dim=np.array([self.k + 1, 1 + self.k + self.n_assets], np.int64),
                        name=f"portfolio_n{self.n_assets}")

    def thetas(self, seed, count):
        return np.random.default_rng(seed).standard_normal((count, self.dim_theta))


# ------------------------------------------------ the paper's workload families
def _sparse_uniform(rng, m, n, density):
    """m x n pattern with about density m n entries (flat positions drawn
    uniformly, repeats merged), values U[0, 1]; CSR."""
    k = int(rng.binomial(m * n, density)) if m * n > 0 else 0
    flat = np.unique(rng.integers(0, m * n, size=k, dtype=np.int64))   # sorted, no repeats
    rows = flat // n
    rp = np.zeros(m + 1, dtype=np.int64)
    rp[1:] = np.cumsum(np.bincount(rows, minlength=m))
    return rp, (flat % n).astype(np.int32), rng.random(flat.size)


def fisher_market(seed, buyers=100, goods=5000, density=0.2, supply=0.25):
    """Fisher market equilibrium in the conic form of the paper's appendix:
    variables [X (buyers x goods, row by row), (p_i, t_i) per buyer],
    min -sum_i w_i p_i  s.t.  sum_i X_ij = b_j,  t_i = sum_j U_ij X_ij,
    (p_i, 1, t_i) in K_exp (p_i <= log t_i),  X >= 0.
    U has the given density with U[0,1] entries (a buyer left without any good
    gets one, else t_i = 0 and the problem is infeasible), w ~ U[0,1],
    b_j = supply.
    Rows: goods clearing and buyer utilities (ZERO), then one EXP block of
    three rows per buyer (its middle row has no entries and h = -1).  No
    planted optimum: the oracle's solution is the reference."""
    rng = np.random.default_rng(seed)
    m, n = buyers, goods
    urp, uci, uval = _sparse_uniform(rng, m, n, density)
    empty = np.flatnonzero(np.diff(urp) == 0)
    if empty.size:   # a buyer with no good of positive utility makes t_i = 0 (infeasible)
        ur = np.repeat(np.arange(m, dtype=np.int64), np.diff(urp))
        urp, uci, uval = csr_from_coo(m, n, np.concatenate([ur, empty]),
                                      np.concatenate([uci, rng.integers(0, n, empty.size)]),
                                      np.concatenate([uval, rng.uniform(0.5, 1.0, empty.size)]))
    w = rng.random(m)
    nx = m * n
    N = nx + 2 * m
    rows, cols, vals = [], [], []
    # goods j: sum_i X_ij = b_j
    i_idx = np.repeat(np.arange(m, dtype=np.int64), n)
    j_idx = np.tile(np.arange(n, dtype=np.int64), m)
    rows.append(j_idx), cols.append(i_idx * n + j_idx), vals.append(np.ones(nx))
    # buyer i: sum_j U_ij X_ij - t_i = 0
    ur = np.repeat(np.arange(m, dtype=np.int64), np.diff(urp))
    rows.append(n + ur), cols.append(ur * n + uci), vals.append(uval)
    rows.append(n + np.arange(m)), cols.append(nx + 2 * np.arange(m) + 1), vals.append(-np.ones(m))
    # exp block of buyer i: rows (p_i, [none], t_i)
    base = n + m + 3 * np.arange(m)
    rows.append(base), cols.append(nx + 2 * np.arange(m)), vals.append(np.ones(m))
    rows.append(base + 2), cols.append(nx + 2 * np.arange(m) + 1), vals.append(np.ones(m))
    M = n + 4 * m
    rp, ci, v = csr_from_coo(M, N, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    h = np.zeros(M)
    h[:n] = supply
    h[base + 1] = -1.0
    c = np.zeros(N)
    c[nx + 2 * np.arange(m)] = -w
    return Instance(n=N, m=M, n_box=0, row_ptr=rp, col=ci, val=v, c=c, h=h,
                    l=np.zeros(0), u=np.zeros(0),
                    xcone_type=np.array([NONNEG, FREE], np.int32),
                    xcone_dim=np.array([nx, 2 * m], np.int64),
                    rcone_type=np.array([ZERO] + [EXP] * m, np.int32),
                    rcone_dim=np.array([n + m] + [3] * m, np.int64),
                    name=f"fisher_m{m}_n{n}",
                    meta=dict(buyers=m, goods=n, u_nnz=int(uval.size), w=w, supply=supply,
                              u_row_ptr=urp, u_col=uci, u_val=uval))


def lasso(seed, rows=10_000, cols=100_000, density=1e-4, form="soc_rows", balance=False):
    """Lasso min ||A x - b||^2 + lambda ||x||_1 in the SOCP form of the paper's
    appendix: variables [w, r, y (rows), x1 (cols), x2 (cols)],
    min 2 r + lambda 1^T (x1 + x2)  s.t.  w = 1,  y - A x1 + A x2 = -b,
    ((w + r)/sqrt 2, (w - r)/sqrt 2, y) in SOC(rows + 2),  x1, x2 >= 0.
    form "soc_rows": the cone constraint as rows+2 rows of G (the appendix's
    form); "rsoc_rows": the same rows written as (w, r, y) in the rotated cone
    (RSOC: 2 w r >= ||y||^2), the same set; "rsoc_x": (w, r, y) is a rotated
    x block, so the rows are only the 1 + rows equalities.
    balance=True fixes w to alpha = ||b|| / sqrt 2 instead of 1 and puts 2 alpha
    on r in the objective: (alpha w, r / alpha, y) is in the rotated cone
    exactly when (w, r, y) is, so the problem and its x1, x2, y are unchanged,
    while w and r (about ||y||^2 / 2 at the optimum) are brought to the same
    scale; meta["alpha"] holds the factor (1 without balancing).
    A has the given density with U[0,1] entries; b = A x~ + 1e-6, x~ ~ N(0,1)
    with half of its entries set to zero; lambda = ||A^T b||_inf.  No planted
    optimum."""
    rng = np.random.default_rng(seed)
    m, n = rows, cols
    arp, aci, aval = _sparse_uniform(rng, m, n, density)
    xt = rng.standard_normal(n)
    xt[rng.permutation(n)[: n // 2]] = 0.0
    b = csr_matvec(arp, aci, aval, xt) + 1e-6
    lam = float(np.abs(csr_rmatvec(arp, aci, aval, b, n)).max()) if n else 0.0
    if form not in ("soc_rows", "rsoc_rows", "rsoc_x"):
        raise ValueError(form)
    N = 2 + m + 2 * n
    M = 1 + m + (0 if form == "rsoc_x" else m + 2)
    # rows in order, columns ascending within each row: w = 1; then per row i
    # of A: y_i, -A_i on x1, +A_i on x2; then the cone rows
    s2 = 1.0 / np.sqrt(2.0)
    alen = np.diff(arp)
    if form == "soc_rows":
        cone_c, cone_v, cone_len = [0, 1, 0, 1], [s2, s2, s2, -s2], [2, 2]
    elif form == "rsoc_rows":
        cone_c, cone_v, cone_len = [0, 1], [1.0, 1.0], [1, 1]
    else:
        cone_c, cone_v, cone_len = [], [], []
    row_len = np.concatenate([[1], 1 + 2 * alen, cone_len,
                              np.ones(m if form != "rsoc_x" else 0, np.int64)]).astype(np.int64)
    rp = np.zeros(M + 1, dtype=np.int64)
    rp[1:] = np.cumsum(row_len)
    ci = np.empty(rp[-1], dtype=np.int32)
    v = np.empty(rp[-1])
    ci[0], v[0] = 0, 1.0
    ys = rp[1:1 + m]                                    # first entry of row 1 + i
    ci[ys], v[ys] = 2 + np.arange(m), 1.0
    ar = np.repeat(np.arange(m, dtype=np.int64), alen)
    pos1 = ys[ar] + 1 + (np.arange(arp[-1], dtype=np.int64) - arp[:-1][ar])
    ci[pos1], v[pos1] = 2 + m + aci, -aval
    pos2 = pos1 + alen[ar]
    ci[pos2], v[pos2] = 2 + m + n + aci, aval
    del ar, pos1, pos2
    if form != "rsoc_x":
        c0 = rp[1 + m]
        ci[c0:c0 + len(cone_c)], v[c0:c0 + len(cone_c)] = cone_c, cone_v
        tail = rp[3 + m:3 + 2 * m]
        ci[tail], v[tail] = 2 + np.arange(m), 1.0
    alpha = float(np.linalg.norm(b) / np.sqrt(2.0)) if balance and m else 1.0
    h = np.zeros(M)
    h[0] = alpha
    h[1:1 + m] = -b
    c = np.zeros(N)
    c[1] = 2.0 * alpha
    c[2 + m:] = lam
    return Instance(n=N, m=M, n_box=0, row_ptr=rp, col=ci, val=v, c=c, h=h,
                    l=np.zeros(0), u=np.zeros(0),
                    xcone_type=np.array([RSOC if form == "rsoc_x" else FREE, NONNEG], np.int32),
                    xcone_dim=np.array([2 + m, 2 * n], np.int64),
                    rcone_type=np.array([ZERO] if form == "rsoc_x" else
                                        [ZERO, RSOC if form == "rsoc_rows" else SOC], np.int32),
                    rcone_dim=np.array([1 + m] if form == "rsoc_x" else [1 + m, m + 2], np.int64),
                    name=f"lasso_m{m}_n{n}" + ("" if form == "soc_rows" else "_" + form)
                    + ("_balanced" if balance else ""),
                    meta=dict(rows=m, cols=n, a_nnz=int(aval.size), lam=lam, b=b, alpha=alpha,
                              a_row_ptr=arp, a_col=aci, a_val=aval))


def logistic(seed, samples=100_000, features=10_000, density=1e-3, l1=0.01, w_density=0.1,
             noise=0.1):
    """Sparse L1-regularised logistic regression as an exponential-cone
    program: min sum_i log(1 + exp(-y_i a_i^T w)) + l1 ||w||_1 over w in R^p,
    for N samples (the loss summed, not averaged: with the average, l1 = 0.01
    exceeds every component of the loss gradient at w = 0 on this data and the
    solution is w = 0).  With w = w+ - w- (w+, w- >= 0) and per sample an
    epigraph variable t_i, log(1 + e^z) <= t holds exactly when
    e^-t + e^(z-t) <= 1, i.e. when some u, v satisfy
        (-t_i, 1, u_i) in K_exp,  (z_i - t_i, 1, v_i) in K_exp,  u_i + v_i <= 1,
    with z_i = -y_i a_i^T w and K_exp = cl{(r, s, t): s > 0, s e^(r/s) <= t}
    (Appendix A.2's order).
    Variables: [w+ (p), w- (p), then (t_i, u_i, v_i) per sample], n = 2p + 3N.
    Rows: N rows 1 - u_i - v_i >= 0 (NONNEG), then per sample two EXP blocks
    of three rows each (their middle rows have no entries and h = -1), so
    m = 7N and 2N exponential cones, whose dual variables take the dual
    exponential projection.  c = (l1 on w+ and w-, 1 on each t_i).
    Data: A (N x p) with Bernoulli(density) pattern and N(0,1) values, a
    planted w* with w_density nonzeros N(0,1), labels y_i =
    sign(a_i^T w* + noise eps_i) (0 -> +1).  No planted optimum: the
    reference objective comes from a tight oracle solve."""
    rng = np.random.default_rng(seed)
    N, p = samples, features
    arp, aci, aval = bernoulli_csr(rng, N, p, density)
    wstar = np.where(rng.random(p) < w_density, rng.standard_normal(p), 0.0)
    score = csr_matvec(arp, aci, aval, wstar) + noise * rng.standard_normal(N)
    lab = np.where(score >= 0.0, 1.0, -1.0)
    n = 2 * p + 3 * N
    m = 7 * N
    i = np.arange(N, dtype=np.int64)
    ct, cu, cv = 2 * p + 3 * i, 2 * p + 3 * i + 1, 2 * p + 3 * i + 2
    base = N + 6 * i
    alen = np.diff(arp)
    ar = np.repeat(i, alen)
    ya = lab[ar] * aval
    rows = np.concatenate([i, i, base, base + 2, base[ar] + 3, base[ar] + 3, base + 3, base + 5])
    cols = np.concatenate([cu, cv, ct, cu, aci.astype(np.int64), p + aci.astype(np.int64), ct, cv])
    vals = np.concatenate([-np.ones(N), -np.ones(N), -np.ones(N), np.ones(N), -ya, ya,
                           -np.ones(N), np.ones(N)])
    rp, ci, v = csr_from_coo(m, n, rows, cols, vals)
    h = np.zeros(m)
    h[:N] = -1.0
    h[base + 1] = -1.0
    h[base + 4] = -1.0
    c = np.zeros(n)
    c[:2 * p] = l1
    c[ct] = 1.0
    return Instance(n=n, m=m, n_box=0, row_ptr=rp, col=ci, val=v, c=c, h=h,
                    l=np.zeros(0), u=np.zeros(0),
                    xcone_type=np.array([NONNEG, FREE], np.int32),
                    xcone_dim=np.array([2 * p, 3 * N], np.int64),
                    rcone_type=np.array([NONNEG] + [EXP] * (2 * N), np.int32),
                    rcone_dim=np.array([N] + [3] * (2 * N), np.int64),
                    name=f"logistic_N{N}_p{p}",
                    meta=dict(samples=N, features=p, l1=l1, labels=lab, w_star=wstar,
                              a_row_ptr=arp, a_col=aci, a_val=aval, a_nnz=int(aval.size)))


def rsoc_min_sum(seed, k=5, form="x"):
    """min u + v over the rotated cone 2 u v >= ||w||^2 (u, v >= 0) with w
    fixed to a seeded w0 ~ N(0, 1)^k.  form "x": x = (u, v, w) is a rotated x
    block and k equality rows fix w; form "rows": x is free, the rows
    (u, v, w) of the identity form a rotated row block and k more rows fix w.
    Optimum u = v = ||w0|| / sqrt 2, objective sqrt 2 ||w0||; meta holds w0."""
    rng = np.random.default_rng(seed)
    w0 = rng.standard_normal(k)
    n = k + 2
    c = np.zeros(n)
    c[:2] = 1.0
    fix_r = np.arange(k, dtype=np.int64)
    fix_c = 2 + np.arange(k, dtype=np.int64)
    if form == "x":
        rp, ci, v = csr_from_coo(k, n, fix_r, fix_c, np.ones(k))
        return Instance(n=n, m=k, n_box=0, row_ptr=rp, col=ci, val=v, c=c, h=w0.copy(),
                        l=np.zeros(0), u=np.zeros(0),
                        xcone_type=np.array([RSOC], np.int32), xcone_dim=np.array([n], np.int64),
                        rcone_type=np.array([ZERO], np.int32), rcone_dim=np.array([k], np.int64),
                        name=f"rsoc_x_{k}", meta=dict(w0=w0))
    rows = np.concatenate([np.arange(n), n + fix_r])
    cols = np.concatenate([np.arange(n), fix_c])
    rp, ci, v = csr_from_coo(n + k, n, rows, cols, np.ones(n + k))
    h = np.concatenate([np.zeros(n), w0])
    return Instance(n=n, m=n + k, n_box=0, row_ptr=rp, col=ci, val=v, c=c, h=h,
                    l=np.zeros(0), u=np.zeros(0),
                    xcone_type=np.array([FREE], np.int32), xcone_dim=np.array([n], np.int64),
                    rcone_type=np.array([RSOC, ZERO], np.int32), rcone_dim=np.array([n, k], np.int64),
                    name=f"rsoc_rows_{k}", meta=dict(w0=w0))

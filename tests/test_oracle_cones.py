"""Pins of the oracle's cone projections (CPU only).

SOC: Section 3 Theorem 1 (proof in Appendix A.1).  EXP: Theorem 3 and the
Remark of Appendix A.2.  Each projection is pinned by facts that do not come
from the oracle itself: the textbook formula that Theorem 1 reduces to when
D = I, the closed-form cases, the Moreau characterisation (Lemma
moreau_decomp: p = Proj_C(v) iff p in C, v - p in the polar of C and
<p, v - p> = 0), and a brute-force 1-D distance search over the boundary rays
of the exponential cone."""
import numpy as np
import pytest

from helpers import kexp_dual_violation, kexp_violation, load_golden, soc_violation

NONNEG, SOC, EXP, EXP_DUAL, ZERO, FREE = 2, 3, 4, 5, 0, 1


def textbook_soc(v):
    t, x = v[0], v[1:]
    nx = np.linalg.norm(x)
    if nx <= t:
        return v.copy()
    if nx <= -t:
        return np.zeros_like(v)
    a = 0.5 * (t + nx)
    return np.concatenate([[a], a * x / nx])


# ------------------------------------------------------------------- SOC
@pytest.mark.parametrize("k", [1, 2, 3, 5, 10, 64, 257])
def test_soc_unscaled_is_textbook(orc, k):
    rng = np.random.default_rng(100 + k)
    for _ in range(200):
        v = rng.standard_normal(k) * 10 ** rng.uniform(-3, 3)
        p, case = orc.proj_soc(v)
        q = textbook_soc(v)
        assert np.allclose(p, q, rtol=1e-13, atol=1e-14 * np.linalg.norm(v)), (v, p, q, case)
        # a uniform D = alpha I leaves the cone and hence the projection unchanged
        p2, _ = orc.proj_soc(v, np.full(k, 10 ** rng.uniform(-2, 2)))
        assert np.allclose(p2, q, rtol=1e-12, atol=1e-13 * np.linalg.norm(v))


def test_soc_case_1_polar_goes_to_zero(orc):
    rng = np.random.default_rng(1)
    for k in (2, 4, 9):
        for _ in range(50):
            d = 10 ** rng.uniform(-1, 1, k)
            x = rng.standard_normal(k - 1)
            u = np.concatenate([[np.linalg.norm(x) + rng.uniform(0.01, 1)], x])  # u in K
            v = -u / d                                   # v in -D^-1 K, the polar of D K
            p, case = orc.proj_soc(v, d)
            assert case == 1 and np.all(p == 0.0)


def test_soc_case_2_inside_is_identity(orc):
    rng = np.random.default_rng(2)
    for k in (2, 4, 9):
        for _ in range(50):
            d = 10 ** rng.uniform(-1, 1, k)
            x = rng.standard_normal(k - 1)
            u = np.concatenate([[np.linalg.norm(x) + rng.uniform(0.01, 1)], x])
            v = d * u                                    # v in D K
            p, case = orc.proj_soc(v, d)
            assert case == 2 and np.array_equal(p, v)


def test_soc_case_3_hand_example(orc):
    g = load_golden("soc_t0_hand.json")
    p, case = orc.proj_soc(np.array(g["v"]), np.array(g["d"]))
    assert case == g["case"]
    assert np.allclose(p, g["proj"], rtol=1e-15, atol=0)


def moreau_soc_ok(v, d, p, tol):
    """p = Proj_{D K}(v) iff D^-1 p in K, -D (v - p) in K, <p, v - p> = 0."""
    q = v - p
    sc = max(1.0, np.linalg.norm(v))
    return (soc_violation(p / d) <= tol * sc / d.min()
            and soc_violation(-d * q) <= tol * sc * d.max()
            and abs(p @ q) <= tol * sc * sc)


@pytest.mark.parametrize("k", [2, 3, 4, 10, 37, 100])
def test_soc_scaled_moreau_certificate(orc, k):
    rng = np.random.default_rng(300 + k)
    cases = set()
    for _ in range(300):
        v = rng.standard_normal(k) * 10 ** rng.uniform(-2, 2)
        d = 10 ** rng.uniform(-1.5, 1.5, k)
        u = rng.random()
        if u < 0.2:
            v[0] = 0.0                                   # exercise case 3
        elif u < 0.35:                                   # inside D K (case 2)
            v[0] = 1.5 * np.linalg.norm(v[1:] * d[0] / d[1:])
        elif u < 0.5:                                    # inside the polar (case 1)
            v[0] = -1.5 * np.linalg.norm(v[1:] * d[1:] / d[0])
        p, case = orc.proj_soc(v, d)
        cases.add(case)
        assert moreau_soc_ok(v, d, p, 1e-11), (v, d, p, case)
        # SOC is self-dual, so (D K)^* = D^-1 K and Moreau gives
        # Proj_{DK}(v) - Proj_{D^-1 K}(-v) = v
        p2, _ = orc.proj_soc(-v, 1.0 / d)
        assert np.allclose(p - p2, v, rtol=1e-10, atol=1e-10 * np.linalg.norm(v))
    if k > 1:
        assert {1, 2, 3, 4} <= cases


def test_soc_idempotent_and_nonexpansive(orc):
    rng = np.random.default_rng(7)
    for _ in range(300):
        k = int(rng.integers(2, 20))
        d = 10 ** rng.uniform(-1, 1, k)
        a = rng.standard_normal(k)
        b = rng.standard_normal(k)
        pa, _ = orc.proj_soc(a, d)
        pb, _ = orc.proj_soc(b, d)
        ppa, _ = orc.proj_soc(pa, d)
        assert np.allclose(ppa, pa, rtol=1e-12, atol=1e-12)
        assert np.linalg.norm(pa - pb) <= np.linalg.norm(a - b) * (1 + 1e-12) + 1e-14


# ------------------------------------------------------------------- EXP
_GRID = np.sinh(np.linspace(-7.25, 7.25, 20001))   # rho in about [-700, 700]


def brute_dist_exp(v, d, dual=False):
    """Distance from v to D K_exp (or D K_exp^*), brute force.  A point that
    meets the cone's defining inequality is at distance 0; any other point's
    nearest cone point lies on the boundary, which is the union of the rays
    alpha w(rho) and one flat face, so its distance is the smaller of the
    distance to the face and the minimum over rho of the distance to a ray
    (1-D grid search + bounded refinement)."""
    if (kexp_dual_violation(v / d) if dual else kexp_violation(v / d)) == 0.0:
        return 0.0
    if not dual:
        face = np.array([min(v[0], 0.0), 0.0, max(v[2], 0.0)])       # {(r,0,t): r<=0<=t}
        ray = lambda rho: d * np.array([rho, 1.0, np.exp(rho)])
    else:
        face = np.array([0.0, max(v[1], 0.0), max(v[2], 0.0)])       # {(0,s,t): s,t>=0}
        ray = lambda rho: d * np.array([-1.0, rho - 1.0, np.exp(-rho)])

    def dist(rho):
        w = ray(rho)
        a = max(v @ w, 0.0) / (w @ w)
        return np.linalg.norm(v - a * w)

    grid = _GRID
    if not dual:
        W = d[None, :] * np.stack([grid, np.ones_like(grid), np.exp(grid)], axis=1)
    else:
        W = d[None, :] * np.stack([-np.ones_like(grid), grid - 1.0, np.exp(-grid)], axis=1)
    a_ = np.maximum(W @ v, 0.0) / np.einsum("ij,ij->i", W, W)
    vals = np.linalg.norm(v[None, :] - a_[:, None] * W, axis=1)
    i = int(np.argmin(vals))
    a, b = grid[max(i - 1, 0)], grid[min(i + 1, grid.size - 1)]
    g = (np.sqrt(5.0) - 1.0) / 2.0                  # golden-section refinement
    c1, c2 = b - g * (b - a), a + g * (b - a)
    f1, f2 = dist(c1), dist(c2)
    for _ in range(200):
        if f1 <= f2:
            b, c2, f2 = c2, c1, f1
            c1 = b - g * (b - a)
            f1 = dist(c1)
        else:
            a, c1, f1 = c1, c2, f2
            c2 = a + g * (b - a)
            f2 = dist(c2)
    return min(np.linalg.norm(v - face), f1, f2, vals[i], np.linalg.norm(v))


def test_exp_closed_cases(orc):
    rng = np.random.default_rng(11)
    for _ in range(300):
        d = 10 ** rng.uniform(-1, 1, 3)
        rho, a = rng.standard_normal(), rng.uniform(0.1, 2)
        # case 1: strictly inside D K_exp
        u = a * np.array([rho, 1.0, np.exp(rho) * rng.uniform(1.01, 3)])
        p, case = orc.proj_exp(d * u, d)
        assert case == 1 and np.array_equal(p, d * u)
        # case 2: inside the polar cone -D^-1 K_exp^*
        w = a * np.array([-1.0, rho - 1.0, np.exp(-rho) * rng.uniform(1.01, 3)])
        p, case = orc.proj_exp(-w / d, d)
        assert case == 2 and np.all(p == 0.0)
        # case 3: r0 <= 0, s0 <= 0 outside both cones -> (r0, 0, t0^+)
        v = np.array([-abs(rng.standard_normal()), -abs(rng.standard_normal()),
                      rng.standard_normal()])
        p, case = orc.proj_exp(v, d)
        if case == 3:
            assert np.array_equal(p, [v[0], 0.0, max(v[2], 0.0)])
        else:
            assert case in (1, 2)


def test_exp_brute_force_distance(orc):
    rng = np.random.default_rng(12)
    seen = set()
    for _ in range(400):
        v = rng.standard_normal(3) * 10 ** rng.uniform(-1, 1, 3)
        d = 10 ** rng.uniform(-0.7, 0.7, 3)
        p, case = orc.proj_exp(v, d)
        seen.add(case)
        sc = max(1.0, np.linalg.norm(v))
        assert brute_dist_exp(p / d, np.ones(3)) <= 1e-9 * sc / d.min()
        db = brute_dist_exp(v, d)
        assert np.linalg.norm(v - p) <= db + 1e-11 * sc, (v, d, p, case)
    assert seen == {1, 2, 3, 4}


def test_exp_moreau_certificate(orc):
    """p = Proj_{D K}(v) iff D^-1 p in K_exp, -D (v - p) in K_exp^*, <p, v-p> = 0.
    Membership is measured as a brute-force distance to the cone, which stays
    well conditioned where the cone's defining inequality is not."""
    rng = np.random.default_rng(13)
    ones = np.ones(3)
    for _ in range(300):
        v = rng.standard_normal(3) * 10 ** rng.uniform(-1, 1, 3)
        d = 10 ** rng.uniform(-0.7, 0.7, 3)
        p, case = orc.proj_exp(v, d)
        q = v - p
        sc = max(1.0, np.linalg.norm(v))
        assert abs(p @ q) <= 1e-10 * sc * sc
        assert brute_dist_exp(p / d, ones) <= 1e-9 * sc / d.min()
        assert brute_dist_exp(-d * q, ones, dual=True) <= 1e-9 * sc * d.max(), (v, d, p, case)


def test_exp_dual_projection(orc):
    """Remark of Appendix A.2, pinned against the dual cone directly."""
    rng = np.random.default_rng(14)
    ones = np.ones(3)
    for _ in range(300):
        v = rng.standard_normal(3) * 10 ** rng.uniform(-1, 1, 3)
        d = 10 ** rng.uniform(-0.7, 0.7, 3)
        p, _ = orc.proj_exp_dual(v, d)
        sc = max(1.0, np.linalg.norm(v))
        assert brute_dist_exp(p / d, ones, dual=True) <= 1e-9 * sc / d.min()
        # the polar of D K^* is -D^-1 K, i.e. -D (v - p) in K_exp
        assert brute_dist_exp(-d * (v - p), ones) <= 1e-9 * sc * d.max()
        assert abs(p @ (v - p)) <= 1e-10 * sc * sc
        db = brute_dist_exp(v, d, dual=True)
        assert np.linalg.norm(v - p) <= db + 1e-11 * sc


def test_exp_extreme_inputs_stay_finite(orc):
    rng = np.random.default_rng(15)
    for _ in range(20000):
        v = rng.standard_normal(3) * 10 ** rng.uniform(-4, 4, 3)
        d = 10 ** rng.uniform(-2.5, 2.5, 3)
        p, _ = orc.proj_exp(v, d)
        q, _ = orc.proj_exp_dual(v, d)
        assert np.all(np.isfinite(p)) and np.all(np.isfinite(q)), (v, d)
        # never farther from v than the origin is
        assert np.linalg.norm(v - p) <= np.linalg.norm(v) * (1 + 1e-12)


def test_exp_far_brackets_stay_finite(orc):
    """Entries of very different magnitude put a3 or a4 of eq. (lrho_urho) far
    beyond |rho| = 700 (the case met in the large workload's dual exp rows:
    r = -1.7e-178, s = 12.4, t = -5.8e-189).  The projection must stay finite
    and never be farther from v than the origin is."""
    p, _ = orc.proj_exp_dual(np.array([-1.66653501e-178, 1.24179468e1, -5.81330326e-189]),
                             np.array([3.01210793, 0.96024127, 0.39153593]))
    assert np.all(np.isfinite(p))
    rng = np.random.default_rng(18)
    for _ in range(20000):
        v = rng.standard_normal(3) * 10.0 ** rng.uniform(-300, 300, 3)
        d = 10 ** rng.uniform(-3, 3, 3)
        for fn in (orc.proj_exp, orc.proj_exp_dual):
            q, _ = fn(v, d)
            assert np.all(np.isfinite(q)), (v, d)
            assert np.linalg.norm(v - q) <= np.linalg.norm(v) * (1 + 1e-12)


def test_exp_denormal_entries(orc):
    """Entries that are 0 or denormal.  The case-4 interval end a3 = r0 ds/(s0 dr)
    (or a4) was once formed as a product over a product: with s0 = -5e-324 (met
    by a restart candidate of the logistic workload, scales (4.64, 1, 1)) s0 dr
    rounds to 0 and a3 became 0/0.  A projection onto a closed convex set is
    nonexpansive, so replacing the tiny entry by 0 moves the projection by at
    most that entry: every output finite and within |delta| (+ rounding)."""
    p, _ = orc.proj_exp_dual(np.array([0.0, -5e-324, 0.9999999903850852]),
                             np.array([4.644325615449967, 1.0, 1.0]))
    assert np.all(np.isfinite(p)) and abs(p[2] - 0.9999999903850852) <= 1e-15
    rng = np.random.default_rng(19)
    tiny = [5e-324, -5e-324, 1e-310, -1e-310, 1e-300, -1e-300, 0.0, -0.0]
    for _ in range(4000):
        v = rng.standard_normal(3) * 10 ** rng.uniform(-2, 2, 3)
        d = 10 ** rng.uniform(-2, 2, 3)
        k = rng.integers(0, 3, size=rng.integers(1, 3))
        w = v.copy()
        w[k] = rng.choice(tiny, size=k.size)
        w0 = w.copy()
        w0[k] = 0.0
        for fn in (orc.proj_exp, orc.proj_exp_dual):
            q, _ = fn(w, d)
            q0, _ = fn(w0, d)
            assert np.all(np.isfinite(q)), (w, d)
            bound = np.linalg.norm(w - w0) + 1e-14 * max(1.0, np.linalg.norm(w))
            assert np.linalg.norm(q - q0) <= bound, (w, d, q, q0)


def test_exp_idempotent(orc):
    rng = np.random.default_rng(16)
    for _ in range(500):
        v = rng.standard_normal(3) * 3
        d = 10 ** rng.uniform(-1, 1, 3)
        p, _ = orc.proj_exp(v, d)
        pp, _ = orc.proj_exp(p, d)
        assert np.allclose(pp, p, rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------ products
def test_product_projection_is_blockwise(orc):
    """eq. (6): a product of cones projects block by block."""
    rng = np.random.default_rng(17)
    types = [NONNEG, SOC, EXP, ZERO, FREE, EXP_DUAL, SOC]
    dims = [4, 5, 3, 2, 3, 3, 1]
    v = rng.standard_normal(sum(dims))
    d = 10 ** rng.uniform(-1, 1, v.size)
    p = orc.proj_blocks(types, dims, v, d)
    o = 0
    for t, k in zip(types, dims):
        vb, db, pb = v[o:o + k], d[o:o + k], p[o:o + k]
        if t == NONNEG:
            assert np.array_equal(pb, np.maximum(vb, 0))
        elif t == ZERO:
            assert np.all(pb == 0)
        elif t == FREE:
            assert np.array_equal(pb, vb)
        elif t == SOC:
            assert np.array_equal(pb, orc.proj_soc(vb, db)[0])
        elif t == EXP:
            assert np.array_equal(pb, orc.proj_exp(vb, db)[0])
        elif t == EXP_DUAL:
            assert np.array_equal(pb, orc.proj_exp_dual(vb, db)[0])
        o += k
    # the dual flag projects onto the dual cones: ZERO <-> FREE, EXP <-> EXP_DUAL
    pd = orc.proj_blocks(types, dims, v, d, dual=True)
    o = 0
    for t, k in zip(types, dims):
        if t == ZERO:
            assert np.array_equal(pd[o:o + k], v[o:o + k])
        if t == FREE:
            assert np.all(pd[o:o + k] == 0)
        if t == EXP:
            assert np.array_equal(pd[o:o + k], orc.proj_exp_dual(v[o:o + k], d[o:o + k])[0])
        o += k

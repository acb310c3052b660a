"""Pins of the oracle's rotated second-order cone (RSOC: 2 u v >= ||w||^2,
u, v >= 0; the cone of the appendix's Lasso form), checked against facts that
do not go through the map the oracle uses for it:

* projection: Moreau's decomposition characterises P_K(v) for a closed convex
  cone: p in K, p - v in K^* (= K, the cone is self-dual: the polar is -K) and
  <p, p - v> = 0; the cone itself is tested from its definition.  Special
  cases: points of K are fixed, points of -K go to 0, and in two dimensions K
  is the nonnegative quadrant, so the projection is max(v, 0);
* solves: min u + v over 2 u v >= ||w0||^2 has the closed form
  u = v = ||w0|| / sqrt 2 (AM-GM), objective sqrt 2 ||w0||, whether the cone
  constrains the variables or the rows; the Lasso written with the rotated
  cone is the same problem as its SOC form, so both give the same objective
  and the same optimality conditions.
"""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

from helpers import lasso_optimality_errors


def rsoc_violation(p):
    """max(0, ||w||^2 - 2 u v, -u, -v) for p = (u, v, w), from the definition."""
    u, v, w = p[0], p[1], p[2:]
    return max(0.0, float(w @ w - 2.0 * u * v), -u, -v)


def inner_rsoc_point(rng, d):
    w = rng.standard_normal(d - 2)
    u = abs(rng.standard_normal()) + 0.1
    v = (w @ w) / (2.0 * u) + abs(rng.standard_normal()) + 1e-3
    return np.concatenate([[u, v], w])


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("d", [2, 3, 4, 7])
def test_projection_satisfies_moreau(orc, seed, d):
    rng = np.random.default_rng(100 * d + seed)
    for _ in range(20):
        v = rng.standard_normal(d) * 10 ** rng.uniform(-2, 2)
        p = orc.proj_blocks([orc.RSOC], [d], v)
        s = max(1.0, float(np.abs(v).max()))
        assert rsoc_violation(p) <= 1e-12 * s * s
        assert rsoc_violation(p - v) <= 1e-12 * s * s
        assert abs(p @ (p - v)) <= 1e-12 * s * s
        assert np.array_equal(orc.proj_blocks([orc.RSOC], [d], v, dual=True), p)


@pytest.mark.parametrize("d", [3, 5])
def test_projection_special_cases(orc, d):
    rng = np.random.default_rng(d)
    for _ in range(10):
        q = inner_rsoc_point(rng, d)
        assert np.allclose(orc.proj_blocks([orc.RSOC], [d], q), q, rtol=1e-14, atol=1e-14)
        assert np.allclose(orc.proj_blocks([orc.RSOC], [d], -q), 0.0, atol=1e-14)
    v = rng.standard_normal((10, 2))
    for vv in v:
        assert np.allclose(orc.proj_blocks([orc.RSOC], [2], vv), np.maximum(vv, 0.0), atol=1e-15)


def test_projection_mixed_blocks(orc):
    """Other blocks of the product are untouched by the rotated one."""
    rng = np.random.default_rng(3)
    types, dims = [orc.NONNEG, orc.RSOC, orc.SOC, orc.RSOC], [3, 4, 3, 5]
    v = rng.standard_normal(15)
    p = orc.proj_blocks(types, dims, v)
    assert np.array_equal(p[:3], np.maximum(v[:3], 0.0))
    assert np.array_equal(p[7:10], orc.proj_blocks([orc.SOC], [3], v[7:10]))
    assert np.array_equal(p[3:7], orc.proj_blocks([orc.RSOC], [4], v[3:7]))
    assert np.array_equal(p[10:], orc.proj_blocks([orc.RSOC], [5], v[10:]))
    with pytest.raises(ValueError):
        orc.proj_blocks(types, dims, v, d=np.ones(15))


@pytest.mark.parametrize("form", ["x", "rows"])
@pytest.mark.parametrize("seed,k", [(1, 1), (2, 5), (3, 12)])
def test_min_sum_closed_form(orc, form, seed, k):
    inst = I.rsoc_min_sum(seed, k=k, form=form)
    r = orc.solve(inst, orc.default_settings(tol=1e-10, max_iter=400_000))
    assert r["status"] == 0
    w0 = inst.meta["w0"]
    t = np.linalg.norm(w0) / np.sqrt(2.0)
    assert r["pobj"] == pytest.approx(np.sqrt(2.0) * np.linalg.norm(w0), rel=1e-8)
    assert np.allclose(r["x"][:2], [t, t], rtol=1e-6, atol=1e-8)
    assert np.allclose(r["x"][2:], w0, rtol=1e-8, atol=1e-9)
    if form == "rows":
        # the multiplier of the rotated rows lies in the (self-dual) cone
        yb = r["y"][:k + 2]
        assert rsoc_violation(yb) <= 1e-8 * max(1.0, float(yb @ yb))


@pytest.mark.parametrize("form,balance", [("rsoc_rows", False), ("rsoc_x", False), ("rsoc_x", True),
                                          ("soc_rows", True)])
@pytest.mark.parametrize("seed,rows,cols,density", [(1, 5, 40, 0.2), (4, 12, 60, 0.15)])
def test_rotated_lasso_is_the_soc_lasso(orc, form, balance, seed, rows, cols, density):
    """The other forms (and the balanced ones, w fixed to alpha) are the same
    problem: same optimal value, same optimality conditions."""
    a = I.lasso(seed, rows=rows, cols=cols, density=density)
    b = I.lasso(seed, rows=rows, cols=cols, density=density, form=form, balance=balance)
    assert (b.meta["alpha"] != 1.0) == balance
    s = orc.default_settings(tol=1e-9, max_iter=400_000)
    ra, rb = orc.solve(a, s), orc.solve(b, s)
    assert ra["status"] == 0 and rb["status"] == 0
    assert rb["pobj"] == pytest.approx(ra["pobj"], rel=1e-8)
    e = lasso_optimality_errors(b, rb["x"])
    assert e["w"] <= 1e-7 and e["y"] <= 1e-6 and e["cone"] <= 1e-6, e
    assert e["stationary_on"] <= 1e-4 and e["stationary_off"] <= 1e-4, e
    if balance or form == "rsoc_x":
        # the multipliers of y - A x1 + A x2 = -b are the same in every form
        assert np.allclose(rb["y"][1:1 + rows], ra["y"][1:1 + rows], rtol=1e-5, atol=1e-7)
        return
    # the rotated rows' multiplier is that of the SOC form, mapped back:
    # (y_u, y_v) = T (y_a, y_b) with T [[1, 1], [1, -1]] / sqrt 2
    ya = ra["y"][1 + rows:3 + rows]
    yb = rb["y"][1 + rows:3 + rows]
    t = np.array([[1.0, 1.0], [1.0, -1.0]]) / np.sqrt(2.0)
    assert np.allclose(yb, t @ ya, rtol=1e-5, atol=1e-7)


def test_kkt_in_the_callers_form(orc):
    """At the closed-form optimum of the rotated problem, in the caller's
    coordinates, every termination measure is at rounding level."""
    inst = I.rsoc_min_sum(4, k=6, form="x")
    w0 = inst.meta["w0"]
    t = np.linalg.norm(w0) / np.sqrt(2.0)
    x = np.concatenate([[t, t], w0])
    # dual: max <w0, y> s.t. c - G^T y = (1, 1, -y) in the rotated cone,
    # i.e. ||y||^2 <= 2, so y = sqrt 2 w0 / ||w0|| with value sqrt 2 ||w0||
    y = np.sqrt(2.0) * w0 / np.linalg.norm(w0)
    lam = np.array([1.0, 1.0]), -y
    k = orc.kkt(inst, x, y)
    assert k["err_p"] <= 1e-14 and k["err_gap"] <= 1e-14, k
    # c - G^T y = (1, 1, -y) must lie in the rotated cone: 2 >= ||y||^2 = 2
    assert rsoc_violation(np.concatenate(lam)) <= 1e-14
    assert k["err_d"] <= 1e-14, k


def test_oracle_library_rejects_unknown_cone_types(orc):
    """The C library rejects cone codes it does not know (the rotated cone
    only reaches it rewritten as an SOC by the wrapper)."""
    import ctypes
    inst = I.rsoc_min_sum(1, k=3, form="x")
    keep = orc._Keep()
    P = orc._problem(inst, keep)         # the raw description: one type-6 block
    x, y = np.empty(inst.n), np.empty(inst.m)
    info = orc._Info()
    s = orc.default_settings()
    rc = orc._lib().orc_solve(ctypes.byref(P), ctypes.byref(s), None, None, 0.0,
                              x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              ctypes.byref(info), None)
    assert rc == -3
    assert orc.solve(inst)["status"] == 0     # through the wrapper's map

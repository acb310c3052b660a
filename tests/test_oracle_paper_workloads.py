"""Pins of the oracle on the paper's two synthetic workload families (the
appendix's conic forms of the Fisher market and of the Lasso), each checked
against facts that do not go through the oracle's own formulas:

* Fisher market: the allocation the oracle returns must be an equilibrium of
  the Eisenberg-Gale program: goods clear, a buyer holds only goods of the
  best utility per price, and every budget is spent at those prices (the
  price of good j is max_i w_i U_ij / u_i, u_i the buyer's utility).
* Lasso: x = x1 - x2 must satisfy the subgradient condition of
  min ||A x - b||^2 + lambda ||x||_1, and its objective must match a plain
  proximal-gradient (ISTA) solve of the original problem.
"""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

from helpers import fisher_equilibrium_errors, lasso_optimality_errors


def _solve(orc, inst, tol=1e-9):
    r = orc.solve(inst, orc.default_settings(tol=tol, max_iter=400_000))
    assert r["status"] == 0, r["status"]
    return r


@pytest.mark.parametrize("seed,buyers,goods", [(1, 4, 6), (2, 4, 6), (3, 8, 30)])
def test_fisher_market_equilibrium(orc, seed, buyers, goods):
    inst = I.fisher_market(seed, buyers=buyers, goods=goods)
    r = _solve(orc, inst)
    e = fisher_equilibrium_errors(inst, r["x"])
    assert e["clearing"] <= 1e-6 and e["negative"] <= 1e-6 and e["utility"] <= 1e-6
    assert e["log"] <= 1e-5
    assert e["bang_per_buck"] <= 1e-4 and e["budget"] <= 1e-4, e


def _ista(A, b, lam, iters=200_000):
    """Proximal gradient on ||A x - b||^2 + lam ||x||_1, step 1/L."""
    L = 2.0 * np.linalg.norm(A, 2) ** 2
    x = np.zeros(A.shape[1])
    for _ in range(iters):
        g = 2.0 * A.T @ (A @ x - b)
        z = x - g / L
        x_new = np.sign(z) * np.maximum(np.abs(z) - lam / L, 0.0)
        if np.abs(x_new - x).max() <= 1e-15:
            x = x_new
            break
        x = x_new
    return x


@pytest.mark.parametrize("seed,rows,cols,density", [(1, 5, 40, 0.2), (2, 5, 40, 0.2), (4, 12, 60, 0.15)])
def test_lasso_optimality(orc, seed, rows, cols, density):
    inst = I.lasso(seed, rows=rows, cols=cols, density=density)
    r = _solve(orc, inst)
    e = lasso_optimality_errors(inst, r["x"])
    assert e["w"] <= 1e-7 and e["y"] <= 1e-6 and e["cone"] <= 1e-6, e
    assert e["stationary_on"] <= 1e-4 and e["stationary_off"] <= 1e-4, e
    m, n = rows, cols
    A = np.zeros((m, n))
    arp, aci, aval = inst.meta["a_row_ptr"], inst.meta["a_col"], inst.meta["a_val"]
    for i in range(m):
        A[i, aci[arp[i]:arp[i + 1]]] = aval[arp[i]:arp[i + 1]]
    b, lam = inst.meta["b"], inst.meta["lam"]
    f = lambda v: float(np.sum((A @ v - b) ** 2) + lam * np.abs(v).sum())
    fi = f(_ista(A, b, lam))
    assert e["objective"] == pytest.approx(fi, rel=1e-7, abs=1e-9)
    assert r["pobj"] == pytest.approx(fi, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("form", ["soc_rows", "rsoc_rows", "rsoc_x"])
@pytest.mark.parametrize("balance", [False, True])
def test_lasso_rows_are_the_appendix_constraints(form, balance):
    """G z - h, for a random z = (w, r, y, x1, x2), written out from the
    appendix's form: w - alpha; y - A x1 + A x2 + b; then the cone rows
    ((w + r)/sqrt 2, (w - r)/sqrt 2, y), or (w, r, y) for the rotated rows,
    or none when the cone is on x.  Also the cone lists, c, and that every
    row's columns ascend."""
    inst = I.lasso(5, rows=30, cols=400, density=0.02, form=form, balance=balance)
    m, n = 30, 400
    rng = np.random.default_rng(1)
    z = rng.standard_normal(inst.n)
    w, r, y, x1, x2 = z[0], z[1], z[2:2 + m], z[2 + m:2 + m + n], z[2 + m + n:]
    A = np.zeros((m, n))
    arp, aci, aval = inst.meta["a_row_ptr"], inst.meta["a_col"], inst.meta["a_val"]
    for i in range(m):
        A[i, aci[arp[i]:arp[i + 1]]] = aval[arp[i]:arp[i + 1]]
    al, b = inst.meta["alpha"], inst.meta["b"]
    want = [[w - al], y - A @ x1 + A @ x2 + b]
    s2 = 1.0 / np.sqrt(2.0)
    if form == "soc_rows":
        want.append([(w + r) * s2, (w - r) * s2])
        want.append(y)
    elif form == "rsoc_rows":
        want.append([w, r])
        want.append(y)
    want = np.concatenate(want)
    G = np.zeros((inst.m, inst.n))
    for i in range(inst.m):
        cols = inst.col[inst.row_ptr[i]:inst.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
        G[i, cols] = inst.val[inst.row_ptr[i]:inst.row_ptr[i + 1]]
    assert np.allclose(G @ z - inst.h, want, rtol=1e-14, atol=1e-12)
    assert inst.c[1] == 2.0 * al and np.all(inst.c[2 + m:] == inst.meta["lam"]) and inst.c[0] == 0.0
    assert (al == 1.0) != balance or al == pytest.approx(np.linalg.norm(b) / np.sqrt(2.0))
    cone = {"soc_rows": I.SOC, "rsoc_rows": I.RSOC}.get(form)
    if cone is None:
        assert list(inst.xcone_type) == [I.RSOC, I.NONNEG] and list(inst.rcone_type) == [I.ZERO]
    else:
        assert list(inst.xcone_type) == [I.FREE, I.NONNEG] and list(inst.rcone_type) == [I.ZERO, cone]

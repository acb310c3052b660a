"""GPU solves of the paper's two synthetic workload families (the appendix's
conic forms of the Fisher market and of the Lasso) against the oracle at
sizes it finishes quickly, and at the paper's smallest Fisher and Lasso
sizes against the equilibrium and optimality conditions, which hold at any
size (see helpers).

Tolerances: both sides stop at a relative KKT error of 1e-8 (the oracle at
1e-9), so objectives agree to 1e-7 relative; the equilibrium and optimality
conditions are derived quantities, held to 1e-6 at 1e-8 and to 1e-4 (1e-3 for
the log and clearing rows, which carry the KKT error of a 5e5-variable
problem times its scale) at the paper size solved to 1e-6."""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

from helpers import fisher_equilibrium_errors, lasso_optimality_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


SMALL = [("fisher_8x30", lambda: I.fisher_market(3, buyers=8, goods=30), fisher_equilibrium_errors),
         ("fisher_20x100", lambda: I.fisher_market(5, buyers=20, goods=100), fisher_equilibrium_errors),
         ("lasso_12x60", lambda: I.lasso(4, rows=12, cols=60, density=0.15), lasso_optimality_errors),
         ("lasso_50x2000", lambda: I.lasso(6, rows=50, cols=2000, density=0.01), lasso_optimality_errors),
         # the same Lasso with (w, r, y) as a rotated x block: only the equality rows
         ("lasso_50x2000_rsoc_x", lambda: I.lasso(6, rows=50, cols=2000, density=0.01, form="rsoc_x"),
          lasso_optimality_errors),
         ("lasso_50x2000_rsoc_x_balanced",
          lambda: I.lasso(6, rows=50, cols=2000, density=0.01, form="rsoc_x", balance=True),
          lasso_optimality_errors)]


@pytest.mark.parametrize("name,maker,check", SMALL, ids=[s[0] for s in SMALL])
def test_paper_workload_matches_oracle(pd, orc, name, maker, check):
    inst = maker()
    say("paper workload", name, inst.n, inst.m, inst.nnz)
    prob = pd.Problem(inst)
    g = prob.solve(pd.settings_default(tol=1e-8))
    prob.close()
    o = orc.solve(inst, orc.default_settings(tol=1e-9, max_iter=2_000_000))
    assert g["status"] == 0 and o["status"] == 0
    assert g["pobj"] == pytest.approx(o["pobj"], rel=1e-7, abs=1e-8)
    e = check(inst, g["x"])
    for k, v in e.items():
        if k != "objective":
            assert v <= 1e-6, (k, v)


def test_fisher_market_paper_size_equilibrium(pd):
    """The paper's smallest Fisher market (100 buyers, 5000 goods, U density
    0.2): solved to 1e-6, the allocation is an equilibrium."""
    inst = I.fisher_market(2025, buyers=100, goods=5000)
    say("fisher paper size", inst.n, inst.m, inst.nnz)
    prob = pd.Problem(inst)
    g = prob.solve(pd.settings_default(tol=1e-6, time_limit=60.0))
    prob.close()
    assert g["status"] == 0, g["status"]
    e = fisher_equilibrium_errors(inst, g["x"])
    say("  iterations", g["iterations"], e)
    assert e["clearing"] <= 1e-3 and e["log"] <= 1e-3
    assert e["negative"] <= 1e-6 and e["utility"] <= 1e-4
    assert e["bang_per_buck"] <= 1e-4 and e["budget"] <= 1e-4


def test_lasso_paper_size_optimality(pd):
    """The paper's smallest Lasso (1e4 x 1e5, A density 1e-4), balanced
    rotated-x form, solved to 1e-6: the subgradient condition of the original
    problem holds at the returned x = x1 - x2."""
    inst = I.lasso(2025, rows=10_000, cols=100_000, form="rsoc_x", balance=True)
    say("lasso paper size", inst.n, inst.m, inst.nnz)
    prob = pd.Problem(inst)
    g = prob.solve(pd.settings_default(tol=1e-6, time_limit=60.0))
    prob.close()
    assert g["status"] == 0, g["status"]
    e = lasso_optimality_errors(inst, g["x"])
    say("  iterations", g["iterations"], e)
    assert e["w"] <= 1e-5 and e["y"] <= 1e-5 and e["cone"] <= 1e-4, e
    assert e["stationary_on"] <= 1e-3 and e["stationary_off"] <= 1e-3, e


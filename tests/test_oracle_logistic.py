"""The exponential-cone logistic-regression workload (CPU only): the
generator's conic form and the oracle's solution of it, pinned against the
original problem min sum log(1 + exp(-y_i a_i^T w)) + l1 ||w||_1 solved
by a bound-constrained quasi-Newton method (scipy), its optimality conditions
and the tightness of the exponential-cone epigraph (Appendix A.2's cone)."""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

from paper_2505_00311_amd import instances as I


def _data(inst):
    M = inst.meta
    N, p = M["samples"], M["features"]
    A = sp.csr_matrix((M["a_val"], M["a_col"], M["a_row_ptr"]), shape=(N, p))
    return N, p, sp.diags(M["labels"]) @ A, M["l1"]


def _direct(inst):
    """The original problem on (w+, w-) >= 0 by L-BFGS-B."""
    N, p, yA, l1 = _data(inst)

    def f(wpm):
        z = -(yA @ (wpm[:p] - wpm[p:]))
        g = -(yA.T @ (1.0 / (1.0 + np.exp(-z))))
        return np.logaddexp(0.0, z).sum() + l1 * wpm.sum(), np.concatenate([g + l1, l1 - g])

    r = so.minimize(f, np.zeros(2 * p), jac=True, method="L-BFGS-B", bounds=[(0, None)] * (2 * p),
                    options=dict(maxiter=20000, ftol=1e-16, gtol=1e-13))
    return r.fun


def test_logistic_structure():
    inst = I.logistic(1, samples=300, features=40, density=0.2)
    N, p = 300, 40
    assert inst.n == 2 * p + 3 * N and inst.m == 7 * N
    assert inst.nnz == 2 * inst.meta["a_nnz"] + 6 * N
    assert list(inst.rcone_dim) == [N] + [3] * (2 * N)
    assert set(np.unique(inst.meta["labels"])) <= {-1.0, 1.0}
    # the middle row of each exponential block is empty with h = -1, so
    # (G x - h) there is the constant 1 of (r, 1, t)
    rl = np.diff(inst.row_ptr)
    mid = N + 6 * np.arange(N) + 1
    assert np.all(rl[mid] == 0) and np.all(inst.h[mid] == -1.0)
    assert np.all(rl[mid + 3] == 0) and np.all(inst.h[mid + 3] == -1.0)


@pytest.mark.parametrize("seed", [20250503, 7])
def test_oracle_solves_the_logistic_problem(orc, seed):
    inst = I.logistic(seed, samples=300, features=30, density=1 / 3)
    r = orc.solve(inst, orc.default_settings(tol=1e-9, max_iter=500_000))
    assert r["status"] == 0
    ref = _direct(inst)
    assert r["pobj"] == pytest.approx(ref, rel=1e-8)
    N, p, yA, l1 = _data(inst)
    x = r["x"]
    w = x[:p] - x[p:2 * p]
    t = x[2 * p::3]
    z = -(yA @ w)
    # the epigraph is tight at the optimum: t_i = log(1 + e^{z_i})
    assert np.abs(t - np.logaddexp(0.0, z)).max() < 1e-6
    # subgradient optimality of the original problem
    g = -(yA.T @ (1.0 / (1.0 + np.exp(-z))))
    assert np.sum(np.abs(w) > 1e-3) >= p // 4      # a non-trivial solution
    nz = np.abs(w) > 1e-6
    assert np.all(np.abs(g[~nz]) <= l1 + 1e-6)
    assert np.allclose(g[nz], -l1 * np.sign(w[nz]), atol=1e-6)

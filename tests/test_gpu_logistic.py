"""GPU parity on the exponential-cone logistic-regression workload (2N
exponential cones on the rows, so every dual step projects onto the dual
exponential cone of the Appendix A.2 Remark): a scaled-down member of the
family (1000 samples x 100 features, 10 entries per row as at full size)
against the oracle, through the C ABI."""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def small():
    return I.logistic(20250503, samples=1000, features=100, density=0.1)


def tiny():
    return I.logistic(20250503, samples=300, features=30, density=1 / 3)


@pytest.fixture(scope="module")
def reference(orc):
    """The oracle run to 1e-9: the reference solution of the tiny member."""
    r = orc.solve(tiny(), orc.default_settings(tol=1e-9, max_iter=500_000))
    assert r["status"] == 0
    return r


def test_logistic_trajectory_200_iterations_fixed_step(pd, orc):
    inst = small()
    say("logistic trajectory", inst.n, inst.m, inst.nnz)
    it = 200
    prob = pd.Problem(inst)
    snaps = np.arange(1, it + 1)
    g = prob.solve(pd.settings_default(max_iter=it, step_mode=1), log_cap=it, snap_iters=snaps)
    prob.close()
    o = orc.solve(inst, orc.default_settings(max_iter=it, step_mode=1), log_cap=it, snap_iters=snaps)
    gl, ol = g["log"], o["log"]
    assert np.array_equal(gl["check_code"], ol["check_code"])
    worst = 0.0
    for i in range(it):
        zg = np.concatenate([gl["snap_x"][i], gl["snap_y"][i]])
        zo = np.concatenate([ol["snap_x"][i], ol["snap_y"][i]])
        worst = max(worst, np.linalg.norm(zg - zo) / max(1.0, np.linalg.norm(zo)))
    say("  worst relative iterate difference", worst)
    assert worst <= 1e-10
    for k in ("beta", "omega"):
        assert np.allclose(gl[k], ol[k], rtol=1e-10, atol=0), k


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_logistic_solve_matches_oracle(pd, orc, reference, precision):
    """FP64 and mixed-precision solves (FP32 products; FP32 products and
    projections) to 1e-6: the oracle's own measures at the GPU answer meet the
    tolerance, and the objective and iterate errors against the oracle's 1e-9
    solution are within what 1e-6 allows."""
    inst = tiny()
    prob = pd.Problem(inst)
    g = prob.solve(pd.settings_default(precision=precision))
    prob.close()
    assert g["status"] == 0
    k = orc.kkt(inst, g["x"], g["y"])
    assert max(k["err_p"], k["err_d"], k["err_gap"]) <= 1.01e-6
    ref = reference["pobj"]
    obj_err = abs(g["pobj"] - ref) / abs(ref)
    x_err = np.abs(g["x"] - reference["x"]).max() / np.abs(reference["x"]).max()
    say("logistic precision", precision, "iterations", g["iterations"], "objective error", obj_err,
        "x error", x_err)
    assert obj_err <= 1e-5
    assert x_err <= 1e-2

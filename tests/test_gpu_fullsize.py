"""Parity at the full sizes the benchmark runs, in the launch configuration it
times (the library's default product layouts: column slabs with the hot-column
front of x for the large instance), against the oracle: 64 fixed-step
iterations (a rounding-stable iteration map; two builds of the oracle that
differ only in FMA contraction stay within 5e-13 of each other here) with
snapshots at iterations 1, 32 and 64 and the decisions of the first check."""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SNAPS = [1, 32, 64]


def say(*a):
    print(*a, flush=True)


def _compare(pd, orc, inst, bound):
    it = SNAPS[-1]
    prob = pd.Problem(inst)
    say("  layouts", prob.layout())
    g = prob.solve(pd.settings_default(max_iter=it, step_mode=1), log_cap=it, snap_iters=SNAPS)
    prob.close()
    o = orc.solve(inst, orc.default_settings(max_iter=it, step_mode=1), log_cap=it, snap_iters=SNAPS)
    gl, ol = g["log"], o["log"]
    assert np.array_equal(gl["check_code"], ol["check_code"]) and ol["check_code"][-1] != 0
    assert gl["check_kkt"][-1] == pytest.approx(ol["check_kkt"][-1], rel=1e-10)
    assert np.allclose(gl["beta"], ol["beta"], rtol=1e-12, atol=0)
    for i, k in enumerate(SNAPS):
        zg = np.concatenate([gl["snap_x"][i], gl["snap_y"][i]])
        zo = np.concatenate([ol["snap_x"][i], ol["snap_y"][i]])
        err = np.linalg.norm(zg - zo) / max(1.0, np.linalg.norm(zo))
        say(f"  iteration {k}: relative iterate difference {err:.3e}")
        assert err <= bound, (k, err)


def test_large_mixed_full_size(pd, orc):
    inst = I.large_mixed(20250502)
    say("large_mixed full size", inst.n, inst.m, inst.nnz)
    _compare(pd, orc, inst, 1e-10)


def test_logistic_full_size(pd, orc):
    inst = I.logistic(20250503)
    say("logistic full size", inst.n, inst.m, inst.nnz)
    _compare(pd, orc, inst, 1e-10)

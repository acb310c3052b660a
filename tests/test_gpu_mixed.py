"""GPU tests of the mixed-precision form: FP32 products with FP64 checks and an
FP64 polish phase, against the FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_00311_amd import instances as I

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("maker", ["small", "lp_soc", "powerlaw"])
def test_fp32_product_within_its_rounding_bound(pd, orc, maker):
    """The FP32 product rounds each value and each x_j to FP32 (relative
    2^-24 each) and forms products and sums in FP64, so entry i is within
    (2^-23 + 2^-47 + k_i 2^-53) sum_j |a_ij x_j| of the exact product, k_i the
    row length; the FP64 product is the oracle's."""
    rng = np.random.default_rng(8)
    if maker == "small":
        inst = I.small_mixed(1)
    elif maker == "lp_soc":
        inst = I.lp_soc_small(20250501)
    else:
        inst = I.large_mixed(4, n=200_000, m=100_000)
    prob = pd.Problem(inst)
    x = rng.standard_normal(inst.n) * 10 ** rng.uniform(-3, 3, inst.n)
    y = rng.standard_normal(inst.m)
    gx = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    gty = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    prob.spmv(dev(x), gx, fp32=True)
    prob.spmv(dev(y), gty, transpose=True, fp32=True)
    torch.cuda.synchronize()
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    ref = orc.spmv(inst.row_ptr, inst.col, inst.val, x)
    absrow = np.zeros(inst.m)
    np.add.at(absrow, rows, np.abs(inst.val * x[inst.col]))
    k = np.diff(inst.row_ptr)
    bound = (2.0 ** -23 + 2.0 ** -47 + k * 2.0 ** -53) * absrow
    got = gx.cpu().numpy()
    assert np.all(np.abs(got - ref) <= bound + 1e-300)
    assert np.abs(got - ref).max() > 0.0      # the FP32 path did run
    order = np.lexsort((rows, inst.col))
    trp = np.concatenate([[0], np.cumsum(np.bincount(inst.col, minlength=inst.n))])
    tref = orc.spmv(trp, rows[order], inst.val[order], y)
    abscol = np.zeros(inst.n)
    np.add.at(abscol, inst.col, np.abs(inst.val * y[rows]))
    kt = np.diff(trp)
    tb = (2.0 ** -23 + 2.0 ** -47 + kt * 2.0 ** -53) * abscol
    assert np.all(np.abs(gty.cpu().numpy() - tref) <= tb + 1e-300)
    prob.close()


MIXED = [("small_mixed_1", lambda: I.small_mixed(1)),
         ("lp_soc_n1000", lambda: I.lp_soc_small(20250501)),
         ("large_mixed_n20000", lambda: I.large_mixed(7, n=20000, m=10000))]


@pytest.mark.parametrize("name,maker", MIXED, ids=[t[0] for t in MIXED])
def test_mixed_solve_reaches_tolerance(pd, orc, name, maker):
    """precision = 1 ends OPTIMAL at 1e-6 as measured by the oracle at its
    answer, and its objective agrees with the FP64 solve and the planted one."""
    inst = maker()
    prob = pd.Problem(inst)
    g = prob.solve(pd.settings_default(precision=1))
    p = prob.solve(pd.settings_default())
    assert g["status"] == 0, g["status"]
    assert g["polish_iter"] != 0
    k = orc.kkt(inst, g["x"], g["y"])
    assert max(k["err_p"], k["err_d"], k["err_gap"]) <= 1.01e-6, k
    # objectives of two 1e-6-KKT answers: see OBJ_REL in test_gpu_batch.py
    assert g["pobj"] == pytest.approx(p["pobj"], rel=3e-5, abs=3e-5)
    if inst.opt is not None:
        assert g["pobj"] == pytest.approx(inst.opt, rel=3e-5, abs=3e-5)
    prob.close()


def test_mixed_polish_switch_by_tolerance(pd, orc):
    """polish_tol = 0 with a huge stall count keeps the FP32 products to the
    end (polish_iter = -1); polish_tol = 1 switches at the first check."""
    inst = I.small_mixed(2)
    prob = pd.Problem(inst)
    a = prob.solve(pd.settings_default(precision=1, polish_tol=0.0, polish_stall=1 << 30, max_iter=640))
    assert a["polish_iter"] == -1
    b = prob.solve(pd.settings_default(precision=1, polish_tol=1.0))
    assert b["polish_iter"] == 64 and b["status"] == 0
    prob.close()


def test_mixed_graph_replay_matches_eager(pd):
    inst = I.large_mixed(7, n=20000, m=10000)
    prob = pd.Problem(inst)
    kw = dict(max_iter=640, precision=1, polish_tol=0.0, polish_stall=1 << 30)
    a = prob.solve(pd.settings_default(use_graph=1, **kw))
    b = prob.solve(pd.settings_default(use_graph=0, **kw))
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])
    prob.close()

"""GPU parity of every product layout (pdcs_set_layout): CSR-stream, row-split
with 4 and 64 lanes, and 1, 2, 4 or 8 column slabs, on both products and in
both precisions, against the FP64 oracle's product; a fixed-step trajectory
under the slab layouts against the oracle's.

Bounds: a layout only changes the order in which a row's products are added,
so the FP64 product is within 1e-14 sum_j |a_ij x_j| of the exact one (the
bound of the default layout's test, above k u for the row lengths here), and
the FP32 product within (2^-23 + 2^-47 + k 2^-53) sum_j |a_ij x_j|, k the row
length (both roundings of a product's inputs, then k FP64 additions)."""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def say(*a):
    print(*a, flush=True)


def layouts(pd):
    return [pd.LAYOUT_STREAM, 4, 64, pd.slabs(1), pd.slabs(2), pd.slabs(4), pd.slabs(8)]


MAKERS = {"small": lambda: I.small_mixed(1),
          "ball_empty_row": lambda: I.ball_socp(1, n=6),
          "lp_soc": lambda: I.lp_soc_small(20250501),
          # power-law columns: G^T rows past 1024 entries take the chunked path
          "powerlaw": lambda: I.large_mixed(4, n=200_000, m=100_000)}


def _check(orc, inst, x, y, gx, gty, fp32):
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    ref = orc.spmv(inst.row_ptr, inst.col, inst.val, x)
    absrow = np.zeros(inst.m)
    np.add.at(absrow, rows, np.abs(inst.val * x[inst.col]))
    order = np.lexsort((rows, inst.col))
    trp = np.concatenate([[0], np.cumsum(np.bincount(inst.col, minlength=inst.n))])
    tref = orc.spmv(trp, rows[order], inst.val[order], y)
    abscol = np.zeros(inst.n)
    np.add.at(abscol, inst.col, np.abs(inst.val * y[rows]))
    if fp32:
        k, kt = np.diff(inst.row_ptr), np.diff(trp)
        b = (2.0 ** -23 + 2.0 ** -47 + k * 2.0 ** -53) * absrow
        bt = (2.0 ** -23 + 2.0 ** -47 + kt * 2.0 ** -53) * abscol
    else:
        b, bt = 1e-14 * absrow, 1e-14 * abscol
    eg = np.abs(gx - ref) - b
    et = np.abs(gty - tref) - bt
    assert np.all(eg <= 1e-300), (int(eg.argmax()), eg.max())
    assert np.all(et <= 1e-300), (int(et.argmax()), et.max())


@pytest.mark.parametrize("maker", list(MAKERS))
def test_every_layout_matches_oracle(pd, orc, maker):
    inst = MAKERS[maker]()
    rng = np.random.default_rng(21)
    x = rng.standard_normal(inst.n) * 10 ** rng.uniform(-2, 2, inst.n)
    y = rng.standard_normal(inst.m)
    prob = pd.Problem(inst)
    gx = torch.empty(max(inst.m, 1), dtype=torch.float64, device="cuda")
    gty = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    xd, yd = dev(x), dev(y)
    for code in layouts(pd):
        say("layout", maker, code, inst.n, inst.m, inst.nnz)
        prob.set_layout(code, code)
        assert prob.layout() == (code, code)
        for fp32 in (False, True):
            gx.fill_(np.nan), gty.fill_(np.nan)
            prob.spmv(xd, gx, fp32=fp32)
            prob.spmv(yd, gty, transpose=True, fp32=fp32)
            torch.cuda.synchronize()
            _check(orc, inst, x, y, gx.cpu().numpy()[:inst.m], gty.cpu().numpy(), fp32)
    prob.close()


def test_slab_product_repeats_bit_for_bit(pd):
    """The slab sums of a row are added in slab order: no run-to-run change."""
    inst = I.large_mixed(4, n=200_000, m=100_000)
    prob = pd.Problem(inst)
    prob.set_layout(pd.slabs(8), pd.slabs(4))
    rng = np.random.default_rng(2)
    xd, yd = dev(rng.standard_normal(inst.n)), dev(rng.standard_normal(inst.m))
    outs = []
    for _ in range(3):
        gx = torch.empty(inst.m, dtype=torch.float64, device="cuda")
        gty = torch.empty(inst.n, dtype=torch.float64, device="cuda")
        prob.spmv(xd, gx)
        prob.spmv(yd, gty, transpose=True)
        torch.cuda.synchronize()
        outs.append((gx.cpu().numpy(), gty.cpu().numpy()))
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])
    prob.close()


def test_layout_codes_checked(pd):
    prob = pd.Problem(I.small_mixed(1))
    g0 = prob.layout()
    for bad in [(3, 0), (0, 128), (pd.slabs(3), 0), (0, -5), (-2, 0)]:
        with pytest.raises(pd.PdcsError):
            prob.set_layout(*bad)
    assert prob.layout() == g0
    prob.set_layout(0, 0)   # the default rule again
    assert prob.layout() == g0
    # the autotuner leaves a caller's layout alone
    prob.set_layout(pd.slabs(2), 8)
    prob.solve(pd.settings_default(max_iter=64, autotune=1))
    assert prob.layout() == (pd.slabs(2), 8)
    prob.close()


@pytest.mark.parametrize("g,gt", [(8, -1), (4, 2)])
def test_trajectory_under_slab_layouts(pd, orc, g, gt):
    """Fixed step, 200 iterations of the scaled-down large workload with the
    slab layouts: same decisions, iterates within the bound of the default
    layout's trajectory test (two FP64 summation orders of the same sums)."""
    inst = I.large_mixed(7, n=20000, m=10000)
    iters = 200
    say("trajectory slabs", g, gt)
    s = pd.settings_default(max_iter=iters, step_mode=1)
    so = orc.default_settings(max_iter=iters, step_mode=1)
    prob = pd.Problem(inst)
    prob.set_layout(pd.slabs(g), pd.slabs(gt) if gt > 0 else gt)
    snaps = np.arange(1, iters + 1)
    r = prob.solve(s, log_cap=iters, snap_iters=snaps)
    o = orc.solve(inst, so, log_cap=iters, snap_iters=snaps)
    prob.close()
    gl, ol = r["log"], o["log"]
    assert np.array_equal(gl["attempts"], ol["attempts"])
    assert np.array_equal(gl["check_code"], ol["check_code"])
    errs = [np.linalg.norm(np.concatenate([gl["snap_x"][i] - ol["snap_x"][i],
                                           gl["snap_y"][i] - ol["snap_y"][i]]))
            / max(1.0, np.linalg.norm(np.concatenate([ol["snap_x"][i], ol["snap_y"][i]])))
            for i in range(iters)]
    say("  worst relative iterate difference", max(errs))
    assert max(errs) <= 1e-8

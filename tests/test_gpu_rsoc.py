"""GPU parity of the rotated second-order cone (PDCS_CONE_RSOC) against the
oracle, which handles the cone with its own map (in its Python wrapper, from
the definition of the cone); the library maps the problem on the host at
creation and the points at the boundary.

Tolerances: projections as the SOC projection tests (1e-12 of the block's
norm: one extra rounding per rotated entry on each side); products within
1e-13 of sum |G| |x| (the map adds a few roundings of the two rows or columns
it mixes); solves as the other solve tests (both sides at a relative KKT error
of 1e-8 / 1e-9, objectives to 1e-7); a fixed-step trajectory within 1e-8 of
the iterate norm (as the slab trajectory test: the GPU and the oracle round
the mapped entries of G differently, (a + b) r against a r + b r)."""
import numpy as np
import pytest

from paper_2505_00311_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def say(*a):
    print(*a, flush=True)


RSOC, SOC, FREE, NONNEG = I.RSOC, I.SOC, I.FREE, I.NONNEG


def mixed_cones(rng, nblk=300):
    types, dims = [], []
    for _ in range(nblk):
        t = int(rng.choice([0, 2, 3, 6, 6, 6, 4]))
        if t == 4:
            k = 3
        elif t in (3, 6):
            k = int(rng.choice([2, 3, 5, 31, 64, 65, 257, 1500]))
        else:
            k = int(rng.integers(1, 20))
        types.append(t), dims.append(k)
    return types, dims


@pytest.mark.parametrize("dual", [False, True])
def test_project_matches_oracle(pd, orc, dual):
    rng = np.random.default_rng(11)
    types, dims = mixed_cones(rng)
    v = np.concatenate([rng.standard_normal(k) * 10 ** rng.uniform(-2, 2) for k in dims])
    say("project rsoc", dual, v.size)
    ref = orc.proj_blocks(types, dims, v, dual=dual)
    vd = dev(v)
    pd.project(types, dims, vd, dual=dual)
    cones = pd.Cones(types, dims)
    vc = dev(v)
    cones.project(vc, dual=dual)
    torch.cuda.synchronize()
    got, gotc = vd.cpu().numpy(), vc.cpu().numpy()
    cones.close()
    assert np.array_equal(got, gotc)
    o = 0
    for t, k in zip(types, dims):
        sc = max(1.0, np.linalg.norm(v[o:o + k]))
        err = np.abs(got[o:o + k] - ref[o:o + k]).max() / sc
        assert err <= 1e-12, (t, k, err)
        o += k


def test_project_rejects_scaling(pd):
    v = dev(np.ones(4))
    with pytest.raises(pd.PdcsError):
        pd.project([RSOC], [4], v, d_dev=dev(np.ones(4)))
    cones = pd.Cones([RSOC], [4])
    with pytest.raises(pd.PdcsError):
        cones.project(v, d_dev=dev(np.ones(4)))
    cones.close()
    with pytest.raises(pd.PdcsError):
        pd.project([RSOC], [1], dev(np.ones(1)))


def test_products_are_the_callers_matrix(pd, orc):
    """pdcs_spmv of a problem with rotated blocks is the product with the
    caller's G: both maps are undone at the boundary."""
    inst = I.lasso(3, rows=40, cols=300, density=0.05, form="rsoc_rows")
    # rotated x blocks as well: the Lasso's x with its free part as one block
    # (w, r) rotated and the rest free
    inst.xcone_type = np.array([RSOC, FREE, NONNEG], np.int32)
    inst.xcone_dim = np.array([2, int(inst.xcone_dim[0]) - 2, int(inst.xcone_dim[1])], np.int64)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(inst.n), rng.standard_normal(inst.m)
    prob = pd.Problem(inst)
    gx = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    gty = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    xd, yd = dev(x), dev(y)
    rows = np.repeat(np.arange(inst.m), np.diff(inst.row_ptr))
    absG = np.zeros(inst.m)
    np.add.at(absG, rows, np.abs(inst.val * x[inst.col]))
    absGt = np.zeros(inst.n)
    np.add.at(absGt, inst.col, np.abs(inst.val * y[rows]))
    ref = orc.spmv(inst.row_ptr, inst.col, inst.val, x)
    order = np.lexsort((rows, inst.col))
    trp = np.concatenate([[0], np.cumsum(np.bincount(inst.col, minlength=inst.n))])
    tref = orc.spmv(trp, rows[order], inst.val[order], y)
    for fp32 in (False, True):
        prob.spmv(xd, gx, fp32=fp32)
        prob.spmv(yd, gty, transpose=True, fp32=fp32)
        torch.cuda.synchronize()
        tol = 1e-6 if fp32 else 1e-13
        assert np.all(np.abs(gx.cpu().numpy() - ref) <= tol * absG.max()), fp32
        assert np.all(np.abs(gty.cpu().numpy() - tref) <= tol * absGt.max()), fp32
    # the inputs are not changed by the map
    assert np.array_equal(xd.cpu().numpy(), x) and np.array_equal(yd.cpu().numpy(), y)
    prob.close()


@pytest.mark.parametrize("form", ["x", "rows"])
@pytest.mark.parametrize("seed,k", [(1, 1), (3, 12)])
def test_min_sum_matches_oracle_and_closed_form(pd, orc, form, seed, k):
    inst = I.rsoc_min_sum(seed, k=k, form=form)
    say("rsoc min sum", form, seed, k)
    prob = pd.Problem(inst)
    g = prob.solve(pd.settings_default(tol=1e-9))
    xo = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    yo = torch.empty(inst.m, dtype=torch.float64, device="cuda")
    gd = prob.solve(pd.settings_default(tol=1e-9), x_out=xo, y_out=yo)
    kk = prob.kkt(xo, yo)
    prob.close()
    o = orc.solve(inst, orc.default_settings(tol=1e-9, max_iter=400_000))
    assert g["status"] == 0 and o["status"] == 0
    w0 = inst.meta["w0"]
    assert g["pobj"] == pytest.approx(np.sqrt(2.0) * np.linalg.norm(w0), rel=1e-7)
    assert g["pobj"] == pytest.approx(o["pobj"], rel=1e-7)
    assert np.allclose(g["x"], o["x"], rtol=1e-5, atol=1e-7)
    # device outputs are mapped like host outputs, and pdcs_kkt reads the
    # caller's form
    assert np.array_equal(xo.cpu().numpy(), g["x"]) and np.array_equal(yo.cpu().numpy(), g["y"])
    assert gd["iterations"] == g["iterations"]
    ko = orc.kkt(inst, g["x"], g["y"])
    for key in ("err_p", "err_d", "err_gap"):
        assert kk[key] <= 1e-8 and ko[key] <= 1e-8, (key, kk[key], ko[key])
    assert kk["pobj"] == pytest.approx(ko["pobj"], rel=1e-12)


def test_rotated_lasso_runs_the_soc_lasso(pd):
    """The library's map turns the rotated Lasso into exactly the hand-written
    SOC form (same rows, same entries, same bits): same iterations, the same
    x, and y equal up to T on the two rotated rows."""
    a = I.lasso(6, rows=50, cols=2000, density=0.01)
    b = I.lasso(6, rows=50, cols=2000, density=0.01, form="rsoc_rows")
    s = pd.settings_default(tol=1e-8)
    pa, pb = pd.Problem(a), pd.Problem(b)
    ra, rb = pa.solve(s), pb.solve(s)
    pa.close(), pb.close()
    assert ra["iterations"] == rb["iterations"]
    assert np.array_equal(ra["x"], rb["x"])
    m = 50
    keep = np.ones(a.m, bool)
    keep[1 + m:3 + m] = False
    assert np.array_equal(ra["y"][keep], rb["y"][keep])
    r = 1.0 / np.sqrt(2.0)
    ya = ra["y"][1 + m:3 + m]
    assert np.allclose(rb["y"][1 + m:3 + m], [(ya[0] + ya[1]) * r, (ya[0] - ya[1]) * r],
                       rtol=1e-15, atol=1e-300)


def test_rotated_lasso_trajectory(pd, orc):
    """Fixed step, 150 iterations with snapshots, starting from a point: the
    starting point, the snapshots and the output all pass through the map."""
    inst = I.lasso(4, rows=12, cols=60, density=0.15, form="rsoc_rows")
    iters = 150
    rng = np.random.default_rng(9)
    x0, y0 = rng.standard_normal(inst.n), rng.standard_normal(inst.m)
    s = pd.settings_default(max_iter=iters, step_mode=1)
    so = orc.default_settings(max_iter=iters, step_mode=1)
    snaps = np.arange(1, iters + 1)
    prob = pd.Problem(inst)
    r = prob.solve(s, x0=x0, y0=y0, log_cap=iters, snap_iters=snaps)
    prob.close()
    o = orc.solve(inst, so, x0=x0, y0=y0, log_cap=iters, snap_iters=snaps)
    gl, ol = r["log"], o["log"]
    assert np.array_equal(gl["check_code"], ol["check_code"])
    errs = [np.linalg.norm(np.concatenate([gl["snap_x"][i] - ol["snap_x"][i],
                                           gl["snap_y"][i] - ol["snap_y"][i]]))
            / max(1.0, np.linalg.norm(np.concatenate([ol["snap_x"][i], ol["snap_y"][i]])))
            for i in range(iters)]
    say("  worst relative iterate difference", max(errs))
    assert max(errs) <= 1e-8
    assert np.allclose(r["x"], o["x"], rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("dropout", [0, 1])
def test_batch_with_rotated_instances(pd, orc, dropout):
    """With dropout = 1 the instances still running are handed to problems
    of their own; their answers must still come back in the caller's form."""
    insts = [I.rsoc_min_sum(2, k=5, form="x"), I.lasso(1, rows=5, cols=40, density=0.2),
             I.rsoc_min_sum(5, k=3, form="rows"),
             I.lasso(4, rows=12, cols=60, density=0.15, form="rsoc_rows")]
    bt = pd.Batch(insts)
    rs = bt.solve(pd.settings_default(tol=1e-8, batch_dropout=dropout))
    bt.close()
    for inst, r in zip(insts, rs):
        say("batch", inst.name, r["status"], r["iterations"])
        o = orc.solve(inst, orc.default_settings(tol=1e-9, max_iter=400_000))
        assert r["status"] == 0 and o["status"] == 0
        assert r["pobj"] == pytest.approx(o["pobj"], rel=1e-7, abs=1e-8)
        k = orc.kkt(inst, r["x"], r["y"])
        assert max(k["err_p"], k["err_d"], k["err_gap"]) <= 2e-8, k


def test_rotated_cone_errors(pd):
    inst = I.rsoc_min_sum(1, k=3, form="x")
    with pytest.raises(pd.PdcsError):
        pd.Problem(inst, from_device=True)        # the map needs host arrays
    bad = I.rsoc_min_sum(1, k=3, form="rows")
    bad.rcone_type = np.array([RSOC, SOC], np.int32)
    pd.Problem(bad).close()                       # valid: RSOC(5) + SOC(3)
    bad.rcone_type = np.array([RSOC, RSOC, SOC], np.int32)
    bad.rcone_dim = np.array([1, 4, 3], np.int64)
    with pytest.raises(pd.PdcsError):
        pd.Problem(bad)                           # a rotated cone needs d >= 2

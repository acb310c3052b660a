"""Pins of the oracle's problem-level functions (CPU only): termination
measures (Section 5 eq. (PDCS_terminate_tolerance)), one PDHG step (Section
2.1 eq. (5)), the diagonal rescaling (Section 3) and the full Algorithm 1."""
import itertools

import numpy as np
import pytest

from helpers import instance_from_dense, load_golden
from paper_2505_00311_amd import instances as I


# ------------------------------------------------------------------ KKT
def _golden_instance(cs):
    return instance_from_dense(cs["n"], cs["m"], cs["n_box"], cs["G"], cs["c"], cs["h"],
                               cs["l"], cs["u"], cs["xcones"], cs["rcones"])


def test_kkt_hand_examples(orc):
    g = load_golden("kkt_hand.json")
    for cs in g["cases"]:
        inst = _golden_instance(cs)
        k = orc.kkt(inst, np.array(cs["x"]), np.array(cs["y"]))
        for key in ("err_p", "err_d", "err_gap", "pobj", "dobj"):
            assert k[key] == pytest.approx(cs[key], rel=1e-15, abs=1e-15), (cs["note"], key)


@pytest.mark.parametrize("maker", [
    lambda: I.small_mixed(0), lambda: I.small_mixed(3, box_kind="finite"),
    lambda: I.lp_soc_small(20250501), lambda: I.large_mixed(5, n=3000, m=1500)])
def test_kkt_zero_at_planted_optimum(orc, maker):
    inst = maker()
    k = orc.kkt(inst, inst.x_star, inst.y_star)
    assert max(k["err_p"], k["err_d"], k["err_gap"]) < 1e-12
    assert k["pobj"] == pytest.approx(inst.opt, rel=1e-12, abs=1e-12)


def test_kkt_responds_to_perturbations(orc):
    inst = I.small_mixed(1)
    rng = np.random.default_rng(0)
    base = orc.kkt(inst, inst.x_star, inst.y_star)
    # moving y off the optimum breaks dual feasibility or the gap
    for eps in (1e-4, 1e-2):
        y = inst.y_star + eps * rng.standard_normal(inst.m)
        k = orc.kkt(inst, inst.x_star, y)
        assert max(k["err_d"], k["err_gap"]) > max(base["err_d"], base["err_gap"]) + eps * 1e-3
    # scaling x by 2 leaves x in its cone but breaks G x - h in K_d^* or the gap
    k = orc.kkt(inst, 2.0 * inst.x_star, inst.y_star)
    assert max(k["err_p"], k["err_gap"]) > 1e-3


# ------------------------------------------------------------ one PDHG step
def test_onepdhg_hand_example(orc):
    g = load_golden("onepdhg_2x2.json")
    pr = g["problem"]
    inst = instance_from_dense(pr["n"], pr["m"], pr["n_box"], pr["G"], pr["c"], pr["h"], [], [],
                               pr["xcones"], pr["rcones"])
    xh, yh = orc.onepdhg(inst, np.array(g["x"]), np.array(g["y"]), g["tau"], g["sigma"])
    assert np.allclose(xh, g["x_hat"], rtol=1e-15, atol=1e-15)
    assert np.allclose(yh, g["y_hat"], rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("name", ["alg1_fixed_2x2.json", "alg1_adaptive_2x2.json"])
def test_algorithm1_worked_examples(orc, name):
    """Four or five iterations of Algorithm 1 on a 2x2 problem, worked out by
    hand (tests/golden/, every intermediate written out): the PDHG step, the
    step acceptance and next step size (adaptive example: a rejection, then
    growth and reduction steps), the reflection parameter (two shrinks, then
    a growth from below 1), the reflected Halpern weights (k+1)/(k+2) and
    1/(k+2), the eta-weighted average, the candidate choice, the restart with
    its primal weight, and the first iteration after it.  A wrong Halpern
    weight or reflection, an unweighted average, another step-size count, a
    missing beta growth factor or an inverted primal-weight ratio each change
    these values (checked by planting each mistake in a copy of the oracle)."""
    g = load_golden(name)
    pr, st = g["problem"], dict(g["settings"])
    inst = instance_from_dense(pr["n"], pr["m"], pr["n_box"], pr["G"], pr["c"], pr["h"], [], [],
                               pr["xcones"], pr["rcones"])
    omega0 = st.pop("omega0")
    its = g["iterations"]
    res = orc.solve(inst, orc.default_settings(**st), omega0=omega0, log_cap=len(its),
                    snap_iters=[r["iteration"] for r in its])
    log = res["log"]
    assert res["iterations"] == len(its) and res["status"] == 1   # iteration limit
    for i, r in enumerate(its):
        assert log["attempts"][i] == r["attempts"], (i, "attempts")
        for key in ("eta_used", "beta", "omega"):
            assert log[key][i] == pytest.approx(r[key], rel=1e-13), (i, key)
        assert np.allclose(log["snap_x"][i], r["x"], rtol=1e-12, atol=1e-14), (i, "x")
        assert np.allclose(log["snap_y"][i], r["y"], rtol=1e-12, atol=1e-14), (i, "y")
    ck = g["check"]
    j = ck["after_iteration"] - 1
    assert log["check_code"][j] == ck["code"]
    kc = ck["kkt_average"] if ck["chosen"] else ck["kkt_current"]
    assert log["check_kkt"][j] == pytest.approx(kc, rel=1e-12)
    assert all(log["check_code"][i] == 0 for i in range(j))
    assert log["check_code"][len(its) - 1] & 8            # the final check stops the solve
    assert res["eta"] == pytest.approx(its[-1]["eta_next"], rel=1e-12)
    # the first iteration after the restart starts from the chosen candidate
    # with the new primal weight
    assert its[j + 1]["omega"] == pytest.approx(ck["omega_after"], rel=1e-15)


def test_onepdhg_fixed_point_at_optimum(orc):
    """A saddle point is a fixed point of eq. (5) for any step sizes."""
    inst = I.small_mixed(2)
    for tau, sigma in ((0.1, 0.1), (0.5, 0.02), (0.01, 2.0)):
        xh, yh = orc.onepdhg(inst, inst.x_star, inst.y_star, tau, sigma)
        assert np.allclose(xh, inst.x_star, atol=1e-11)
        assert np.allclose(yh, inst.y_star, atol=1e-11)


# ---------------------------------------------------------------- scaling
def test_scaling_ruiz_equilibrates(orc):
    """Enough Ruiz passes drive every row and column infinity norm of E G F to 1."""
    inst = I.small_mixed(4, n=60, m=30, density=0.3)
    s = orc.default_settings(ruiz_iters=60, pock_chambolle=0)
    e, f = orc.scaling(inst, s)
    A = np.abs(inst.dense()) * e[:, None] * f[None, :]
    rows = A.max(axis=1)
    cols = A.max(axis=0)
    assert np.allclose(rows[rows > 0], 1.0, atol=1e-6)
    assert np.allclose(cols[cols > 0], 1.0, atol=1e-6)


def test_scaling_pock_chambolle_closed_form(orc):
    """With no Ruiz pass, one alpha=1 Pock-Chambolle pass on a rank-one |u v^T|
    gives e_i = (|u_i| sum|v|)^-1/2, f_j = (|v_j| sum|u|)^-1/2."""
    rng = np.random.default_rng(3)
    u = rng.uniform(0.5, 3, 5) * rng.choice([-1, 1], 5)
    v = rng.uniform(0.5, 3, 7) * rng.choice([-1, 1], 7)
    G = np.outer(u, v)
    inst = instance_from_dense(7, 5, 7, G, np.ones(7), np.ones(5), [-1] * 7, [1] * 7, [],
                               [[2, 5]])
    e, f = orc.scaling(inst, orc.default_settings(ruiz_iters=0, pock_chambolle=1))
    assert np.allclose(e, 1 / np.sqrt(np.abs(u) * np.abs(v).sum()), rtol=1e-14)
    assert np.allclose(f, 1 / np.sqrt(np.abs(v) * np.abs(u).sum()), rtol=1e-14)


def test_scaling_empty_rows_and_columns_keep_one(orc):
    G = np.array([[0.0, 4.0, 0.0], [0.0, 0.0, 0.0]])
    inst = instance_from_dense(3, 2, 3, G, np.ones(3), np.ones(2), [-1] * 3, [1] * 3, [],
                               [[2, 2]])
    e, f = orc.scaling(inst, orc.default_settings(ruiz_iters=1, pock_chambolle=0))
    assert e[1] == 1.0 and f[0] == 1.0 and f[2] == 1.0
    assert e[0] == 0.5 and f[1] == 0.5          # one pass: 1/sqrt(4) each


# ------------------------------------------------------------------ solve
def _check_solution(inst, r, tol):
    assert r["status"] == 0
    assert max(r["err_p"], r["err_d"], r["err_gap"]) <= tol
    assert r["pobj"] == pytest.approx(inst.opt, rel=10 * tol, abs=10 * tol)


@pytest.mark.parametrize("seed", range(6))
def test_solve_recovers_planted_objective(orc, seed):
    inst = I.small_mixed(seed)
    r = orc.solve(inst)
    _check_solution(inst, r, 1e-6)


def test_solve_lp_soc_small_workload(orc):
    inst = I.lp_soc_small(20250501)
    r = orc.solve(inst)
    _check_solution(inst, r, 1e-6)


def test_solve_tight_tolerance(orc):
    inst = I.small_mixed(1)
    r = orc.solve(inst, orc.default_settings(tol=1e-9))
    assert r["status"] == 0
    assert r["pobj"] == pytest.approx(inst.opt, rel=1e-8, abs=1e-8)


def _lp_vertex_enumeration(inst):
    """min c^T x over {G x >= h, l <= x <= u}: best feasible vertex."""
    A = inst.dense()
    n = inst.n
    rows = [(A[i], inst.h[i]) for i in range(inst.m)]
    rows += [(np.eye(n)[j], inst.l[j]) for j in range(n)]
    rows += [(-np.eye(n)[j], -inst.u[j]) for j in range(n)]
    best = np.inf
    for act in itertools.combinations(range(len(rows)), n):
        M = np.array([rows[i][0] for i in act])
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        x = np.linalg.solve(M, np.array([rows[i][1] for i in act]))
        if all(a @ x >= b - 1e-9 for a, b in rows):
            best = min(best, inst.c @ x)
    return best


@pytest.mark.parametrize("seed", range(5))
def test_solve_tiny_lp_vs_vertex_enumeration(orc, seed):
    inst = I.tiny_lp(seed, n=3, m=3)
    ref = _lp_vertex_enumeration(inst)
    r = orc.solve(inst, orc.default_settings(tol=1e-9))
    assert r["status"] == 0
    assert r["pobj"] == pytest.approx(ref, rel=1e-7, abs=1e-7)


@pytest.mark.parametrize("seed", range(4))
def test_solve_ball_socp_closed_form(orc, seed):
    """min c^T x s.t. ||W (x - x0)|| <= r has x* = x0 - r W^-2 c / ||W^-1 c||."""
    inst = I.ball_socp(seed)
    W, x0, rad = inst.meta["W"], inst.meta["x0"], inst.meta["r"]
    xs = x0 - rad * (inst.c / W ** 2) / np.linalg.norm(inst.c / W)
    r = orc.solve(inst, orc.default_settings(tol=1e-9))
    assert r["status"] == 0
    assert np.allclose(r["x"], xs, atol=1e-6)
    assert r["pobj"] == pytest.approx(inst.c @ xs, rel=1e-8, abs=1e-8)


def test_solve_constant_beta_modes_converge(orc):
    inst = I.small_mixed(3)
    for beta in (0.0, 0.5, 1.0):
        r = orc.solve(inst, orc.default_settings(beta_mode=1, beta_const=beta, max_iter=200000))
        _check_solution(inst, r, 1e-6)


def test_solve_status_codes(orc):
    inst = I.small_mixed(0)
    r = orc.solve(inst, orc.default_settings(max_iter=100))
    assert r["status"] == 1 and r["iterations"] == 100
    r = orc.solve(inst, orc.default_settings(max_iter=0))
    assert r["status"] == 1 and r["iterations"] == 0
    # warm start at the planted optimum terminates before the first iteration
    r = orc.solve(inst, x0=inst.x_star, y0=inst.y_star)
    assert r["status"] == 0 and r["iterations"] == 0
    # a NaN in the data ends in NUMERICAL, not in a crash or a hang
    bad = I.small_mixed(0)
    bad.c = bad.c.copy()
    bad.c[3] = np.nan
    r = orc.solve(bad, orc.default_settings(max_iter=500))
    assert r["status"] == 3


def test_solve_decision_log_is_consistent(orc):
    inst = I.small_mixed(5)
    s = orc.default_settings(max_iter=400)
    r = orc.solve(inst, s, log_cap=400, snap_iters=[1, 64, 65, 400])
    lg = r["log"]
    assert lg["attempts"].size == 400 and np.all(lg["attempts"] >= 1)
    assert np.all((lg["beta"] >= 0) & (lg["beta"] <= 1)) and np.all(lg["eta_used"] > 0)
    checks = np.nonzero(lg["check_code"])[0] + 1
    # checks every 64 inner iterations (restarts only happen at checks) plus the
    # forced check at the iteration limit
    assert np.all(checks[:-1] % 64 == 0) and checks[-1] == 400
    # first check after the start: k = N >= 0.36 N, so some restart rule fires
    assert (lg["check_code"][63] - 1) // 2 % 4 != 0
    # the snapshot at iteration 65 follows a restart, so it differs from 64's
    assert not np.allclose(lg["snap_x"][1], lg["snap_x"][2])


def test_fixed_step_uses_the_spectral_norm(orc):
    """step_mode 1: eta = step_fixed / ||E G F||_2, the norm from power
    iteration; it can only underestimate the norm, and 100 iterations get
    within a few percent on these matrices."""
    for seed in (0, 3):
        inst = I.small_mixed(seed)
        e, f = orc.scaling(inst)
        sig = np.linalg.norm(inst.dense() * e[:, None] * f[None, :], 2)
        r = orc.solve(inst, orc.default_settings(step_mode=1, max_iter=64))
        est = 0.9 / r["eta"]
        assert est <= sig * (1 + 1e-12) and est >= 0.95 * sig, (est, sig)


@pytest.mark.parametrize("seed", range(3))
def test_fixed_step_solves(orc, seed):
    inst = I.small_mixed(seed)
    r = orc.solve(inst, orc.default_settings(step_mode=1, max_iter=400000))
    _check_solution(inst, r, 1e-6)


def test_solve_without_rows(orc):
    inst = I.box_only()
    r = orc.solve(inst, orc.default_settings(tol=1e-9))
    assert r["status"] == 0 and r["iterations"] > 0
    assert np.allclose(r["x"], inst.x_star, atol=1e-8)


# ------------------------------------------------ the baseline PDHG (plain mode)
def test_plain_pdhg_is_textbook_pdhg(orc):
    """plain_pdhg = 1 without rescaling: the iterates are those of textbook PDHG
    with tau = sigma = 0.9 / ||G||_2 (||G||_2 from an SVD here, by power
    iteration in the oracle), written out below with the box and
    nonnegative-orthant projections of this LP."""
    from paper_2505_00311_amd import instances as I
    inst = I.tiny_lp(7, n=6, m=5)
    G = inst.dense()
    eta = 0.9 / np.linalg.svd(G, compute_uv=False)[0]
    l, u = inst.l, inst.u
    x = np.clip(np.zeros(inst.n), l, u)
    y = np.zeros(inst.m)
    iters = 6
    ref = []
    for _ in range(iters):
        xh = np.clip(x - eta * (inst.c - G.T @ y), l, u)
        yh = np.maximum(y + eta * (inst.h - G @ (2 * xh - x)), 0.0)
        x, y = xh, yh
        ref.append((x.copy(), y.copy()))
    s = orc.default_settings(ruiz_iters=0, pock_chambolle=0, plain_pdhg=1, max_iter=iters,
                             power_iters=500)
    r = orc.solve(inst, s, log_cap=iters, snap_iters=np.arange(1, iters + 1))
    for k in range(iters):
        assert np.allclose(r["log"]["snap_x"][k], ref[k][0], rtol=1e-9, atol=1e-12), k
        assert np.allclose(r["log"]["snap_y"][k], ref[k][1], rtol=1e-9, atol=1e-12), k
    assert np.all(r["log"]["beta"][:iters] == 0.0)
    assert np.allclose(r["log"]["omega"][:iters], 1.0)


def test_plain_pdhg_reaches_the_planted_optimum(orc):
    from paper_2505_00311_amd import instances as I
    inst = I.small_mixed(1)
    r = orc.solve(inst, orc.default_settings(plain_pdhg=1, tol=1e-7, max_iter=2_000_000))
    assert r["status"] == 0
    assert r["pobj"] == pytest.approx(inst.opt, rel=1e-5, abs=1e-5)
    assert r["restarts"] == 0


def test_timing_mode_threads(orc):
    """The OpenMP timing mode runs the same iteration with reductions in
    another order: fixed-step iterates stay within rounding of the
    single-thread ones, and switching back to one thread restores the
    deterministic bits."""
    inst = I.large_mixed(7, n=20000, m=10000)
    s = orc.default_settings(max_iter=128, step_mode=1)
    a = orc.solve(inst, s)
    try:
        orc.set_threads(4)
        assert orc.get_threads() == 4
        b = orc.solve(inst, s)
    finally:
        orc.set_threads(1)
    c = orc.solve(inst, s)
    assert np.array_equal(a["x"], c["x"]) and np.array_equal(a["y"], c["y"])
    za, zb = np.concatenate([a["x"], a["y"]]), np.concatenate([b["x"], b["y"]])
    assert np.linalg.norm(za - zb) <= 1e-8 * np.linalg.norm(za)

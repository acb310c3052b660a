"""Benchmark of the PDCS hot path on one MI355X.

Workload: the large single instance (n = 1e6 variables, m = 5e5 rows,
~1e7 nonzeros with power-law column degrees, rows scaled over 1e-3..1e3; 1e5
box entries, 2e4 SOC blocks, 1e4 exponential-cone row blocks; planted optimum),
generated from a fixed seed.  A step is one check period of Algorithm 1: 64
accepted PDHG iterations (primal pass, SpMV G x^, dual pass, step decision,
SpMV G^T y^, Halpern/average update) followed by the restart/termination check.
The problem is on the device before the timed region starts.

Prints one JSON line (see the repository's benchmark contract).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-6 rel. KKT & PDHG iter/s (plain FP64 vs chosen form), HBM GB/s"
SEED_LARGE = 20250502
SEED_BATCH = 20250504
SEED_FAMILY = 20250505
SEED_FISHER = 20250506
SEED_LASSO = 20250507
HBM_PEAK_GBS = 8000.0
CHECK = 64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(rows, cols, nnz):
    """Algorithmic HBM bytes of one CSR product in FP64: values and column
    indices once (12 B/nnz), row pointers, the output, and x read once."""
    return 12 * nnz + 8 * (rows + 1) + 8 * rows + 8 * cols


def iteration_bytes(n, m, nnz):
    """Algorithmic bytes of one accepted iteration (FP64 path as built): two
    CSR products plus the vector traffic of the fused passes (primal pass: read
    x, G^T y, c, scale; write x^ -- dual pass: read y, G x^, G x, h, scale; write
    y^ -- Halpern/average: read x^, x, x0, G^T y^, G^T y, G^T y0, sum, write x,
    G^T y, sum, and the same on the row side)."""
    primal = 8 * 5 * n
    dual = 8 * 6 * m
    halpern = 8 * 10 * (n + m)
    return spmv_bytes(m, n, nnz) + spmv_bytes(n, m, nnz) + primal + dual + halpern


FP32_ONLY = dict(precision=1, polish_tol=0.0, polish_stall=1 << 30)
FP32_PROJ_ONLY = dict(precision=2, polish_tol=0.0, polish_stall=1 << 30)


def kernel_timing(pdcs, prob, iters, **kw):
    """Per-kernel average durations inside a solve of `iters` iterations from a
    cold start (the timed work again), from HIP events that the library records
    on its solve stream around every step-attempt kernel."""
    r = prob.solve(pdcs.settings_default(max_iter=iters, time_kernels=1, **kw))
    us = {k: 1e3 * r["kernel_ms"][k] / max(1, r["kernel_launches"][k]) for k in pdcs.KERNELS}
    return us, r


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the summary is missing, covers another kernel, or
    the kernel's source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_large_mixed_n1e6.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"<!-- traffic: (\{.*?\}) -->", open(path).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = os.path.join(ROOT, rec["source"])
    if kernel not in rec["kernels"] or not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["sha256"]:
        return None
    return rec["kernels"][kernel]["bytes_per_launch"]


def batched_512_record():
    """The committed record of the batched configuration at its size (512
    instances, 4.5e9 nonzeros; `--config4` reproduces it), or None.  Not
    measured in this run: it takes about seven minutes of GPU time."""
    import re
    path = os.path.join(ROOT, "profiles", "batched_512_instances.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"<!-- record: (\{.*?\}) -->", open(path).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    rec.update({"recorded": True, "measured_in_this_run": False,
                "source": "profiles/batched_512_instances.md",
                "command": "python bench.py --config4 --c4-mode batch --c4-time-limit 420; "
                           "python bench.py --config4 --c4-mode single --c4-stride 16 --c4-time-limit 90"})
    return rec


def exp_fp64_flops():
    """FP64 operations per launch of the 2e5-cone dual exponential projection of
    the logistic workload, from the committed rocprofv3 counter summary (FMA
    counted as two), or None when it is missing or the projection code changed
    since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "exp_projection_logistic.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"<!-- fp64: (\{.*?\}) -->", open(path).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    if not isinstance(rec.get("sources"), dict):
        return None
    for path, sha in rec["sources"].items():
        src = os.path.join(ROOT, path)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != sha:
            return None
    return rec["fp64_flop_per_launch"]


def layout_name(code):
    if code <= -10:
        return f"{-10 - code} column slabs (spmv_slab_kernel)"
    if code == -1:
        return "CSR-stream (spmv_stream_kernel)"
    return f"row-split, {code} lanes per row (spmv_rows_kernel)"


def product_name(kernel, layouts):
    g, gt = layouts
    if kernel == "spmv_g":
        return f"SpMV G~ x^: {layout_name(g)}; slab sums finished in the dual pass"
    return (f"SpMV G~^T y^: {layout_name(gt)}; step decision in the same launch, "
            "slab and long-row chunk sums finished in the Halpern step")


def batched_form(pdcs, instances, torch, count, limit=20.0):
    """Time to 1e-6 of `count` independent planted LP/SOCP instances (n uniform
    in 1e3..2e4, m = n/2, 0.5% density, 20% of the variables in SOC blocks of
    dims 3..50): one batched solve (autotuned products) against solving them one
    after another with the plain single-problem solver, each side under the
    same time limit.  The speedup is taken over the members that reach 1e-6 on
    both sides (the batch's finish time of the last of them against the sum of
    their single solve times), so that a member that fails on both sides does
    not set both times; the shifted geometric means count failures at the
    limit, as the paper counts them."""
    insts = instances.batch_lp_soc(SEED_BATCH, count, n_lo=1000, n_hi=20000)
    nnz = sum(i.nnz for i in insts)
    log(f"batched form: {count} instances, sum n {sum(i.n for i in insts)}, sum nnz {nnz}")
    batch = pdcs.Batch(insts)
    batch.solve(pdcs.settings_default(max_iter=64, autotune=1))   # tune and warm up
    log("  batch created and tuned")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rb = batch.solve(pdcs.settings_default(time_limit=limit, autotune=1))
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    batch.close()
    worst = 0.0
    its_single, t_single, ok_single = [], [], []
    for i, (inst, r) in enumerate(zip(insts, rb)):
        if i % 16 == 0:
            log(f"  one by one: instance {i} of {count}")
        prob = pdcs.Problem(inst)
        prob.solve(pdcs.settings_default(max_iter=64))   # scaling and graph, as for the batch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = prob.solve(pdcs.settings_default(time_limit=limit))
        torch.cuda.synchronize()
        t_single.append(time.perf_counter() - t0)
        its_single.append(rs["iterations"])
        ok_single.append(rs["status"] == 0)
        if rs["status"] == 0 and r["status"] == 0:
            worst = max(worst, abs(r["pobj"] - rs["pobj"]) / max(1.0, abs(rs["pobj"])))
        prob.close()
    ok_b = [r["status"] == 0 for r in rb]
    both = [i for i in range(count) if ok_b[i] and ok_single[i]]
    t_b = max([rb[i]["done_s"] for i in both], default=0.0)
    t_s = sum(t_single[i] for i in both)
    its_b = [r["iterations"] for r in rb]
    # throughput in instance-iterations per second: independent of how many
    # iterations the slowest instance happens to need on each path (the
    # adaptive rule's count moves with the summation order)
    tp_b, tp_s = sum(its_b) / wall_b, sum(its_single) / sum(t_single)
    sgm_b = sgm([rb[i]["done_s"] if ok_b[i] else limit for i in range(count)])
    sgm_s = sgm([t_single[i] if ok_single[i] else limit for i in range(count)])
    log(f"batched: {sum(ok_b)}/{count} optimal, one by one: {sum(ok_single)}/{count} (limit {limit:.0f}s each); "
        f"the {len(both)} optimal on both: batched {t_b:.2f}s vs one by one {t_s:.2f}s; "
        f"instance-iterations/s {tp_b:.0f} vs {tp_s:.0f}; SGM(10) {sgm_b:.2f}s vs {sgm_s:.2f}s")
    return {"workload": f"{count} planted LP/SOCP instances, n in 1e3..2e4, m = n/2, 0.5% density, "
                        f"20% SOC dims 3..50, seed {SEED_BATCH}",
            "sum_nnz": nnz, "time_limit_s": limit,
            "optimal_batched": sum(ok_b), "optimal_one_by_one": sum(ok_single),
            "optimal_both": len(both),
            "batched_s": round(t_b, 3), "one_by_one_s": round(t_s, 3),
            "speedup_time_to_tol": round(t_s / max(t_b, 1e-9), 3),
            "batched_wall_s": round(wall_b, 3), "one_by_one_wall_s": round(sum(t_single), 3),
            "sgm10_batched_s": round(sgm_b, 3), "sgm10_one_by_one_s": round(sgm_s, 3),
            "max_objective_diff_vs_single_rel": worst,
            "iterations_max": max(its_b), "iterations_max_one_by_one": max(its_single),
            "instance_iter_per_s_batched": round(tp_b, 1),
            "instance_iter_per_s_one_by_one": round(tp_s, 1),
            "speedup_iter_throughput": round(tp_b / tp_s, 3)}


# the paper's H100 times for its larger Lasso sizes (rows, cols): 1e-3, 1e-6
PAPER_LASSO_S = {(400_000, 7_000_000): {"1e-3": 120.0, "1e-6": 260.0},
                 (700_000, 7_000_000): {"1e-3": 320.0, "1e-6": 520.0},
                 (750_000, 7_500_000): {"1e-3": 470.0, "1e-6": 600.0}}


def paper_workloads(pdcs, instances, torch, extra_lasso=()):
    """The paper's two synthetic families: the Fisher market (100 buyers, 5000
    goods, U density 0.2) and the Lasso at its two smaller sizes (1e4 x 1e5 and
    7e4 x 7e5, A density 1e-4), solved from cold to 1e-3 and 1e-6.  The Lasso
    takes (w, r, y) as a rotated x block (G holds only the equality rows) with
    w fixed to alpha = ||b|| / sqrt 2 (the same problem: the block is in the
    cone for any alpha); the appendix's w = 1 is also solved at the smaller
    size, to 1e-3 (capped at 30 s).  The paper's H100 times are context, not a
    target.  extra_lasso: further (rows, cols) sizes, balanced, to both
    tolerances (capped at 300 s each)."""
    lasso = lambda rows, bal: instances.lasso(SEED_LASSO, rows=rows, cols=10 * rows, form="rsoc_x", balance=bal)
    cases = [("fisher_market", instances.fisher_market(SEED_FISHER, buyers=100, goods=5000),
              {"1e-3": 15.0, "1e-6": 37.0}, (1e-3, 1e-6), 300.0),
             ("lasso 1e4x1e5", lasso(10_000, True), {"1e-3": 0.071, "1e-6": 0.11}, (1e-3, 1e-6), 60.0),
             ("lasso 7e4x7e5", lasso(70_000, True), {"1e-3": 0.29, "1e-6": 0.84}, (1e-3, 1e-6), 60.0),
             ("lasso 1e4x1e5, w = 1", lasso(10_000, False), {"1e-3": 0.071}, (1e-3,), 30.0)]
    cases += [(f"lasso {r:.2g}x{c:.2g}", (r, c), PAPER_LASSO_S.get((r, c), {}), (1e-3, 1e-6), 300.0)
              for r, c in extra_lasso]
    res = {}
    for name, inst, paper, tols, cap in cases:
        if isinstance(inst, tuple):   # generated only when its turn comes (tens of GB)
            t0 = time.perf_counter()
            inst = instances.lasso(SEED_LASSO, rows=inst[0], cols=inst[1], form="rsoc_x", balance=True)
            log(f"{name}: generated in {time.perf_counter() - t0:.1f}s, G nnz {inst.nnz}")
        prob = pdcs.Problem(inst)
        prob.solve(pdcs.settings_default(max_iter=64))   # scaling and graph
        torch.cuda.synchronize()
        rec = {"n": inst.n, "m": inst.m, "nnz": inst.nnz, "paper_h100_s": paper}
        for tol in tols:
            t0 = time.perf_counter()
            r = prob.solve(pdcs.settings_default(tol=tol, time_limit=cap))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            status = {0: "optimal", 1: "iteration limit", 2: "time limit"}.get(r["status"], str(r["status"]))
            key = f"{tol:.0e}".replace("e-0", "e-")
            rec[key] = {"status": status, "solve_s": round(r["solve_s"], 3), "wall_s": round(wall, 3),
                        "iterations": r["iterations"], "objective": r["pobj"],
                        "kkt": max(r["err_p"], r["err_d"], r["err_gap"])}
            log(f"{name} to {tol:g}: {status}, {r['solve_s']:.2f}s, {r['iterations']} iterations")
        prob.close()
        del inst
        res[name] = rec
    return res


def pdhg_ablation(pdcs, instances, torch, cap_s=30.0):
    """The paper's PDHG-versus-PDCS comparison on synthetic stand-ins for its
    SOC and exponential-cone sets: time and iterations to 1e-6 of Algorithm 1
    and of the baseline PDHG (fixed step 0.9/||G~||_2 on both sides, no
    Halpern step, no restarts; the same rescaling), the baseline capped at
    cap_s seconds."""
    cases = [("lp_soc n=1000", instances.lp_soc_small(20250501)),
             ("large_mixed n=20000 (SOC + exp)", instances.large_mixed(7, n=20000, m=10000)),
             ("fisher_market 100x5000 (exp)", instances.fisher_market(SEED_FISHER, buyers=100, goods=5000))]
    res = []
    for name, inst in cases:
        prob = pdcs.Problem(inst)
        prob.solve(pdcs.settings_default(max_iter=64))
        rec = {"workload": name, "n": inst.n, "m": inst.m, "nnz": inst.nnz}
        for key, kw in (("pdcs", {}), ("pdhg", {"plain_pdhg": 1})):
            torch.cuda.synchronize()
            r = prob.solve(pdcs.settings_default(tol=1e-6, time_limit=cap_s, **kw))
            torch.cuda.synchronize()
            rec[key] = {"status": pdcs.SOLVE_STATUS[r["status"]], "solve_s": round(r["solve_s"], 3),
                        "iterations": r["iterations"],
                        "kkt": max(r["err_p"], r["err_d"], r["err_gap"])}
            log(f"ablation {name} {key}: {rec[key]['status']}, {r['solve_s']:.2f}s, {r['iterations']} iterations")
        if rec["pdhg"]["status"] == "optimal":
            rec["speedup_time"] = round(rec["pdhg"]["solve_s"] / rec["pdcs"]["solve_s"], 2)
        else:
            rec["speedup_time_at_least"] = round(cap_s / rec["pdcs"]["solve_s"], 2)
        prob.close()
        res.append(rec)
    return res


def projection_sweeps(pdcs, torch, total=1_200_000_000, soc_counts=None, exp_counts=None):
    """The projection benchmarks of the paper's Section 4: a random vector
    projected onto m SOC blocks of dimension ceil(total/m) + 1 (D = I), and
    onto a growing number of exponential cones.  Each point: median of 5 HIP-
    event-timed projections on a reused plan, each from a fresh copy of the
    same input; bytes = one read and one write of the vector."""
    # 1 and 10 cones (dimensions 1.2e9 and 1.2e8): grid-level blocks of 512 parts
    soc_counts = soc_counts or [1, 10, 100, 1000, 10_000, 100_000, 1_000_000, 10_000_000]
    exp_counts = exp_counts or [10 ** k for k in range(2, 8)]

    def timed(types, dims):
        n = int(np.sum(dims))
        src = torch.randn(n, dtype=torch.float64, device="cuda")
        v = torch.empty_like(src)
        cones = pdcs.Cones(types, dims)
        ms = []
        for r in range(6):
            v.copy_(src)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            cones.project(v)
            b.record()
            torch.cuda.synchronize()
            if r:
                ms.append(a.elapsed_time(b))
        cones.close()
        del src, v
        torch.cuda.empty_cache()
        t = float(np.median(ms))
        gbs = 16.0 * n / (t * 1e-3) / 1e9
        return {"entries": n, "ms": round(t, 3), "gb_s": round(gbs, 1),
                "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}

    soc = []
    for m in soc_counts:
        d = -(-total // m)
        rec = timed(np.full(m, 3, np.int32), np.full(m, d + 1, np.int64))
        rec.update(cones=m, dim=d + 1)
        soc.append(rec)
        log(f"SOC sweep: {m} cones of dim {d + 1}: {rec['ms']} ms, {rec['gb_s']} GB/s")
    ex = []
    for k in exp_counts:
        rec = timed(np.full(k, 4, np.int32), np.full(k, 3, np.int64))
        rec.update(cones=k)
        ex.append(rec)
        log(f"exp sweep: {k} cones: {rec['ms']} ms, {rec['gb_s']} GB/s")
    return {"soc": soc, "exp": ex, "roofline_ms_soc": round(16.0 * total / (HBM_PEAK_GBS * 1e9) * 1e3, 3)}


def warm_start_form(pdcs, instances, torch, n_assets, n_train, n_test):
    """Learned warm start on the parametric SOC portfolio family (k = 50 factors,
    theta in R^64): batched solves of n_train parameters give the targets, the
    network 64 -> 512 -> 512 -> (n + m + 1) is trained on the GPU, and n_test
    held-out parameters are solved cold and from its predictions."""
    from paper_2505_00311_amd import warmstart as W
    fam = instances.PortfolioFamily(SEED_FAMILY, n_assets=n_assets, k=50)
    tr = fam.thetas(SEED_FAMILY + 1, n_train)
    te = fam.thetas(SEED_FAMILY + 2, n_test)
    t0 = time.perf_counter()
    res, _ = W.solve_family(fam, tr, log=log)
    gen_s = time.perf_counter() - t0
    T = W.targets_of(res)
    del res
    net, norm, hist, train_s = W.train(tr, T, hidden=512, epochs=100, batch=256, lr=1e-3, log=log)
    # the output layer's GEMM on the matrix cores: 256 x (n + m + 1) x 512
    th = torch.randn(256, 64, dtype=torch.float32, device="cuda")
    out = torch.empty(256, net.n_out, dtype=torch.float32, device="cuda")
    net.forward(th, out)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(20):
        net.forward(th, out)
    b.record()
    b.synchronize()
    fwd_ms = a.elapsed_time(b) / 20
    flops = 2.0 * 256 * (64 * 512 + 512 * 512 + 512 * net.n_out)
    cold, cold_s = W.solve_family(fam, te, log=log)
    starts = W.predict(net, norm, te, fam.n, fam.m)
    warm, warm_s = W.solve_family(fam, te, starts=starts, log=log)
    net.close()
    it_c = float(np.mean([r["iterations"] for r in cold]))
    it_w = float(np.mean([r["iterations"] for r in warm]))
    ok = sum(r["status"] == 0 for r in warm)
    log(f"warm start: held-out iterations cold {it_c:.0f} warm {it_w:.0f}; time {cold_s:.2f}s vs {warm_s:.2f}s")
    return {"workload": f"SOC portfolio family, {n_assets} assets, 50 factors, theta in R^64, "
                        f"{n_train} training and {n_test} held-out parameters, seed {SEED_FAMILY}",
            "n": fam.n, "m": fam.m, "network": f"64-512-512-{net.n_out} BF16/FP32-accumulate",
            "training_solves_s": round(gen_s, 2), "training_s": round(train_s, 2),
            "loss_first_last": [hist[0], hist[-1]],
            "held_out_iterations_cold": it_c, "held_out_iterations_warm": it_w,
            "held_out_optimal_warm": ok,
            "cold_s": round(cold_s, 3), "warm_s": round(warm_s, 3),
            "speedup_time_to_tol": round(cold_s / warm_s, 3),
            "forward_ms_batch256": round(fwd_ms, 4),
            "forward_tflops": round(flops / (fwd_ms * 1e-3) / 1e12, 2),
            "mfma_bf16_peak_tflops": 2500.0}


def host_threads():
    """Host threads the oracle's timing mode may use: the box's share
    (OMP_NUM_THREADS when set), else every core."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, int(env)) if env.isdigit() else (os.cpu_count() or 1)


def oracle_rate(inst, iters, threads, **kw):
    """Oracle iterations per second over its first `iters` iterations, setup
    (rescaling, transpose) excluded by subtracting a 0-iteration run."""
    import oracle
    oracle.build(force=False)
    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        oracle.solve(inst, oracle.default_settings(max_iter=0, **kw))
        t1 = time.perf_counter()
        r = oracle.solve(inst, oracle.default_settings(max_iter=iters, **kw))
        t2 = time.perf_counter()
    finally:
        oracle.set_threads(1)
    run = (t2 - t1) - (t1 - t0)
    return r["iterations"] / run, run


def cpu_baseline(inst, iters, gpu_iters_to_tol=None):
    """The oracle as it stands on the first `iters` iterations of the same
    instance: the OpenMP timing mode on the host's threads (the value) and the
    deterministic single-thread mode beside it.  With the GPU's iteration
    count to 1e-6, the oracle's time to tolerance is extrapolated from its
    rate (an estimate: the oracle is not run that long)."""
    threads = host_threads()
    v_all, run_all = oracle_rate(inst, iters, threads)
    v_one, run_one = oracle_rate(inst, iters, 1)
    rec = {"value": round(v_all, 3), "unit": "iter/s", "cores": threads, "kind": "oracle",
           "sample": f"first {iters} PDHG iterations (one check period) of the same instance, "
                     f"setup excluded; {run_all:.1f} s on {threads} host threads (OpenMP timing "
                     f"mode), {run_one:.1f} s on 1 thread",
           "single_thread_value": round(v_one, 3), "host_cpu_count": os.cpu_count()}
    if gpu_iters_to_tol:
        rec["estimated_time_to_tol_s"] = round(gpu_iters_to_tol / v_all, 1)
        rec["estimated_time_to_tol_note"] = (f"estimate: {gpu_iters_to_tol} iterations (the GPU "
                                             f"solve's count to 1e-6) at the measured oracle rate")
    return rec


def small_instance(pdcs, instances, torch, oracle_on=True):
    """The small single instance (n = 1000, m = 500, 1% density, 500 nonneg +
    50 SOC(10) on x; latency-bound): iterations per second, microseconds per
    iteration and time to 1e-6 on the GPU, and the oracle's full solve to 1e-6
    on one host thread beside it."""
    inst = instances.lp_soc_small(20250501)
    prob = pdcs.Problem(inst)
    prob.solve(pdcs.settings_default(max_iter=64))   # scaling and graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = prob.solve(pdcs.settings_default(max_iter=64 * 50, tol=0.0))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ips = r["iterations"] / r["solve_s"]
    t0 = time.perf_counter()
    rt = prob.solve(pdcs.settings_default())
    torch.cuda.synchronize()
    wall_t = time.perf_counter() - t0
    prob.close()
    rec = {"workload": f"lp_soc n={inst.n} m={inst.m} nnz={inst.nnz} (500 nonneg + 50 SOC(10) on x, "
                       "250 equality + 250 inequality rows, seed 20250501)",
           "bound": "latency (five launches per step attempt; 0.29 MB per iteration stays in L2)",
           "iter_per_s": round(ips, 1), "us_per_iteration": round(1e6 / ips, 2),
           "timed_iterations": r["iterations"], "wall_s": round(wall, 3),
           "time_to_tol": {"tol": 1e-6, "status": pdcs.SOLVE_STATUS[rt["status"]],
                           "solve_s": round(rt["solve_s"], 4), "wall_s": round(wall_t, 4),
                           "iterations": rt["iterations"], "objective": rt["pobj"],
                           "planted_objective": inst.opt}}
    if oracle_on:
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        ro = oracle.solve(inst, oracle.default_settings())
        wall_o = time.perf_counter() - t0
        rec["oracle_1_thread"] = {"solve_s_incl_setup": round(wall_o, 3), "iterations": ro["iterations"],
                                  "iter_per_s": round(ro["iterations"] / wall_o, 1),
                                  "status": ro["status"], "objective": ro["pobj"]}
        rec["speedup_time_to_tol_vs_oracle"] = round(wall_o / max(rt["solve_s"], 1e-9), 2)
    log(f"small instance: {ips:.0f} iter/s ({1e6 / ips:.1f} us/iteration); to 1e-6 in "
        f"{rt['solve_s']:.4f}s, {rt['iterations']} iterations")
    return rec


SEED_LOGISTIC = 20250503


def logistic_form(pdcs, instances, torch):
    """The exponential-cone logistic-regression workload (1e5 samples x 1e4
    features, 0.1% density, 2e5 exponential cones on the rows): time to 1e-6 in
    FP64 and in the mixed form, each answer's objective error against the
    oracle's 1e-9 reference (tests/golden/logistic_reference.json), iterations
    per second, and the dual exponential projection of the 2e5 cones timed on
    its own (a projection plan applied to the dual iterate of the solve)."""
    t = time.perf_counter()
    inst = instances.logistic(SEED_LOGISTIC)
    log(f"logistic: n={inst.n} m={inst.m} nnz={inst.nnz} generated in {time.perf_counter() - t:.1f}s")
    ref_path = os.path.join(ROOT, "tests", "golden", "logistic_reference.json")
    ref = json.load(open(ref_path)) if os.path.exists(ref_path) else None
    prob = pdcs.Problem(inst)
    prob.solve(pdcs.settings_default(max_iter=64))
    torch.cuda.synchronize()
    rec = {"workload": f"logistic N=1e5 p=1e4 density 1e-3 l1 0.01, n={inst.n} m={inst.m} "
                       f"nnz={inst.nnz}, {2 * inst.meta['samples']} exp cones on rows, seed {SEED_LOGISTIC}",
           "reference": None if ref is None else {"objective": ref["pobj"], "tol": ref["tol"],
                                                   "iterations": ref["iterations"]}}
    out = {}
    for name, kw in (("fp64", {}), ("mixed", {"precision": 1}), ("mixed_fp32_projections", {"precision": 2})):
        t0 = time.perf_counter()
        r = prob.solve(pdcs.settings_default(time_limit=120.0, **kw))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e = {"status": pdcs.SOLVE_STATUS[r["status"]], "solve_s": round(r["solve_s"], 3),
             "wall_s": round(wall, 3), "iterations": r["iterations"],
             "iter_per_s": round(r["iterations"] / max(r["solve_s"], 1e-9), 1),
             "kkt_max": max(r["err_p"], r["err_d"], r["err_gap"]), "objective": r["pobj"]}
        if ref is not None:
            e["objective_rel_err_vs_oracle"] = abs(r["pobj"] - ref["pobj"]) / abs(ref["pobj"])
        if name != "fp64":
            e["polish_iter"] = r["polish_iter"]
        out[name] = (e, r)
        rec[name] = e
        log(f"logistic {name}: {e['status']} in {e['solve_s']}s, {e['iterations']} iterations, "
            f"objective error {e.get('objective_rel_err_vs_oracle')}")
    rec["mixed_speedup_time_to_tol"] = round(rec["fp64"]["solve_s"] / max(rec["mixed"]["solve_s"], 1e-9), 3)
    rec["mixed_fp32_projections_speedup_time_to_tol"] = round(
        rec["fp64"]["solve_s"] / max(rec["mixed_fp32_projections"]["solve_s"], 1e-9), 3)
    # the 2e5 dual exponential projections alone, on the final dual iterate
    N = inst.meta["samples"]
    y = torch.from_numpy(out["fp64"][1]["y"][N:].copy()).cuda()
    cones = pdcs.Cones(np.full(2 * N, 4, np.int32), np.full(2 * N, 3, np.int64))
    v = torch.empty_like(y)
    ms = []
    for k in range(6):
        v.copy_(y)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        cones.project(v, dual=True)
        b.record()
        torch.cuda.synchronize()
        if k:
            ms.append(a.elapsed_time(b))
    cones.close()
    t_exp = float(np.median(ms))
    rec["dual_exp_projection"] = {"cones": 2 * N, "ms": round(t_exp, 4),
                                  "cones_per_s": round(2 * N / (t_exp * 1e-3), 1),
                                  "input": "the FP64 solve's dual iterate on the exponential rows"}
    fl = exp_fp64_flops()
    if fl is not None:   # ALU-bound work: FP64 operations against the vector peak
        rec["dual_exp_projection"].update({
            "fp64_flop_per_launch": fl, "fp64_tflops": round(fl / (t_exp * 1e-3) / 1e12, 2),
            "fp64_vector_peak_tflops": 78.6,
            "timing_note": "HIP events around one launch (includes the launch gap)"})
    prob.close()
    return rec


def _member(args):
    seed, b, count = args
    from paper_2505_00311_amd import instances
    return instances.batch_member(seed, b, count)


def sgm(times, shift=10.0):
    """Shifted geometric mean SGM(k) of Section 5: (prod (t_i + k))^(1/N) - k."""
    t = np.asarray(times, dtype=np.float64)
    return float(np.exp(np.mean(np.log(t + shift))) - shift)


def config4(args):
    """The batched configuration at its size: `count` independent planted
    LP/SOCP instances (n uniform in 1e3..1e5, m = n/2, 0.5% density, 20% of the
    variables in SOC blocks of dims 3..50; about 4.3e9 nonzeros in all).

    mode "batch": one batch of all of them in the mixed form (FP32 products,
    FP64 checks and polish), product layouts by the autotuner, with a time
    limit; reports the wall time, how many finished, and SGM(10) of the
    instances' finish times (an unfinished instance counts the limit).
    mode "single": every stride-th instance solved alone with the plain FP64
    solver (the same time limit each), the per-instance times and SGM(10) of
    that sample.  Instances are generated on the host by a process pool
    before anything touches the GPU (each member has its own child seed)."""
    import multiprocessing as mp
    from paper_2505_00311_amd import instances
    count, seed = args.c4_count, SEED_BATCH
    sizes = instances.batch_sizes(seed, count)
    idx = list(range(count)) if args.c4_mode == "batch" else list(range(0, count, args.c4_stride))
    t0 = time.perf_counter()
    workers = max(1, min(host_threads(), 16))
    insts = []
    with mp.get_context("fork").Pool(workers) as pool:
        for inst in pool.imap(_member, [(seed, b, count) for b in idx], chunksize=1):
            insts.append(inst)
            if len(insts) % 64 == 0:
                log(f"  generated {len(insts)} of {len(idx)} instances ({time.perf_counter() - t0:.0f}s)")
    gen_s = time.perf_counter() - t0
    nnz = sum(i.nnz for i in insts)
    log(f"config 4 ({args.c4_mode}): {len(insts)} instances, sum nnz {nnz}, generated in {gen_s:.1f}s "
        f"on {workers} processes")
    os.environ.setdefault("PDCS_LOG", "1")   # stage lines of the batch set-up (minutes)
    import torch
    from paper_2505_00311_amd import pdcs
    torch.cuda.set_device(0)
    out = {"metric": METRIC, "mode": args.c4_mode, "data": "synthetic",
           "workload": f"{count} planted LP/SOCP instances (n uniform in 1e3..1e5, m = n/2, 0.5% density, "
                       f"20% SOC dims 3..50, seed {seed}); sum n {int(sizes.sum())}",
           "instances": len(insts), "sum_nnz": nnz, "generate_s": round(gen_s, 1),
           "time_limit_s": args.c4_time_limit}
    if args.c4_mode == "batch":
        t0 = time.perf_counter()
        batch = pdcs.Batch(insts)
        torch.cuda.synchronize()
        out["create_s"] = round(time.perf_counter() - t0, 1)
        log(f"  batch created in {out['create_s']}s")
        del insts
        t0 = time.perf_counter()
        rb = batch.solve(pdcs.settings_default(precision=args.c4_precision, autotune=1, batch_dropout=args.c4_dropout,
                                                 time_limit=args.c4_time_limit,
                                                 log_every=30.0))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        batch.close()
        done = [r["done_s"] if r["status"] == 0 else args.c4_time_limit for r in rb]
        its = [r["iterations"] for r in rb]
        out.update({"form": ("batched, FP32 products + FP64 checks and polish, autotuned layouts" if args.c4_precision
                             else "batched, plain FP64, autotuned layouts"),
                    "wall_s": round(wall, 2), "solve_s": round(rb[0]["solve_s"], 2),
                    "setup_s": round(rb[0]["setup_s"], 2),
                    "optimal": sum(r["status"] == 0 for r in rb),
                    "sgm10_s": round(sgm(done), 3),
                    "iterations_median": int(np.median(its)), "iterations_max": int(max(its)),
                    "finish_s_quantiles": [round(float(q), 2) for q in np.quantile(done, [0.1, 0.5, 0.9, 1.0])],
                    "finish_s": [round(float(t), 3) for t in done], "status": [int(r["status"]) for r in rb],
                    "iterations": [int(i) for i in its]})
    else:
        times, its, ok = [], [], 0
        for k, inst in zip(idx, insts):
            prob = pdcs.Problem(inst)
            prob.solve(pdcs.settings_default(max_iter=64))
            torch.cuda.synchronize()
            r = prob.solve(pdcs.settings_default(time_limit=args.c4_time_limit))
            torch.cuda.synchronize()
            prob.close()
            t = r["solve_s"] if r["status"] == 0 else args.c4_time_limit
            times.append(t), its.append(r["iterations"])
            ok += r["status"] == 0
            log(f"  instance {k} (n {inst.n}, nnz {inst.nnz}): {pdcs.SOLVE_STATUS[r['status']]} in "
                f"{r['solve_s']:.2f}s, {r['iterations']} iterations")
        out.update({"form": "one by one, plain FP64", "sample_stride": args.c4_stride,
                    "sample": idx, "optimal": ok, "times_s": [round(t, 3) for t in times],
                    "iterations": its, "sum_s": round(sum(times), 2), "sgm10_s": round(sgm(times), 3),
                    "sum_s_extrapolated_to_all": round(sum(times) * count / len(times), 1)})
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--layout", default=None,
                    help="product layouts 'G,GT' as pdcs_set_layout codes (default: the library's)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-workloads", action="store_true")
    ap.add_argument("--no-projection-sweeps", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the n = 1000 latency-bound instance")
    ap.add_argument("--no-logistic", action="store_true", help="skip the logistic-regression workload")
    ap.add_argument("--lasso-sizes", default="",
                    help="extra Lasso sizes 'ROWSxCOLS,...' for the paper workloads (the paper's "
                         "larger ones: 400000x7000000,700000x7000000,750000x7500000; each takes "
                         "a minute or more)")
    ap.add_argument("--cpu-iters", type=int, default=64)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=500_000)
    ap.add_argument("--family-assets", type=int, default=20000,
                    help="assets of the warm-start family (0: skip the warm-start measurement)")
    ap.add_argument("--family-train", type=int, default=2048)
    ap.add_argument("--family-test", type=int, default=256)
    ap.add_argument("--batch-count", type=int, default=128,
                    help="instances of the batched-form measurement (0: skip it)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the reference kernel "
                         "for scaling HBM byte counters) and exit")
    ap.add_argument("--config4", action="store_true",
                    help="only the batched configuration at its size (512 instances, ~4.3e9 "
                         "nonzeros; many minutes), printing its own JSON line")
    ap.add_argument("--c4-mode", choices=["batch", "single"], default="batch")
    ap.add_argument("--c4-dropout", type=int, default=2,
                    help="settings.batch_dropout of the batched solve (2: hand stragglers over when the "
                         "batch-wide launches cost 4x their own work)")
    ap.add_argument("--c4-precision", type=int, default=1,
                    help="settings.precision of the batched solve: 0 plain FP64, 1 FP32 products")
    ap.add_argument("--c4-count", type=int, default=512)
    ap.add_argument("--c4-stride", type=int, default=16)
    ap.add_argument("--c4-time-limit", type=float, default=300.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sharded "
              "multi-GPU path is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.config4:   # generates on the host before anything touches the GPU
        config4(args)
        return

    import torch
    from paper_2505_00311_amd import instances
    from paper_2505_00311_amd import pdcs

    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {nb} bytes 5 times")
        return
    t = time.perf_counter()
    inst = instances.large_mixed(SEED_LARGE, n=args.n, m=args.m)
    log(f"generated n={inst.n} m={inst.m} nnz={inst.nnz} in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    prob = pdcs.Problem(inst)
    if args.layout:
        prob.set_layout(*[int(v) for v in args.layout.split(",")])
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t
    log(f"problem created (upload, G^T, plans) in {create_s:.2f}s; product layouts {prob.layout()}")

    # warmup: W check periods (also computes and caches the rescaling)
    prob.solve(pdcs.settings_default(max_iter=CHECK * max(args.warmup, 1)))
    torch.cuda.synchronize()
    log("warmup done")

    # timed: K check periods from a cold start
    K = args.steps
    s = pdcs.settings_default(max_iter=CHECK * K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = prob.solve(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = r["iterations"]
    ips = iters / r["solve_s"]
    ms_per_step = wall / K * 1e3
    log(f"timed {K} steps: {iters} iterations, {r['attempts']} attempts, solve {r['solve_s']:.3f}s "
        f"(wall {wall:.3f}s, setup {r['setup_s']:.3f}s) -> {ips:.1f} iter/s")

    bytes_iter = iteration_bytes(inst.n, inst.m, inst.nnz)
    hbm_gbs = bytes_iter * ips / 1e9

    # per-kernel durations inside the solve; the dominant kernel is the product
    # with the larger summed time
    kus, rk = kernel_timing(pdcs, prob, CHECK * K)
    tot = {k: rk["kernel_ms"][k] for k in pdcs.KERNELS}
    dom = "spmv_g" if tot["spmv_g"] >= tot["spmv_gt"] else "spmv_gt"
    b_dom = spmv_bytes(inst.m, inst.n, inst.nnz) if dom == "spmv_g" else spmv_bytes(inst.n, inst.m, inst.nnz)
    t_dom = kus[dom] * 1e-6
    ach = b_dom / t_dom / 1e9
    log("in-solve kernel averages (us): " + ", ".join(f"{k} {v:.1f}" for k, v in kus.items())
        + f"; event-timed solve {rk['iterations'] / rk['solve_s']:.1f} iter/s")
    dom_name = product_name(dom, prob.layout())

    out = {
        "metric": METRIC,
        "value": round(ips, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"large_mixed n={inst.n} m={inst.m} nnz={inst.nnz} "
                               f"(power-law columns, 1e5 box, 2e4 SOC, 1e4 exp row blocks, seed {SEED_LARGE})",
                   "form": "plain FP64", "step": "64 PDHG iterations + restart/termination check"},
        "hbm_model_gbs": round(hbm_gbs, 1),
        "hbm_model_frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
        "bytes_per_iteration_model": bytes_iter,
        "roofline": {"bound": "hbm", "kernel": dom_name,
                     "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": counter_traffic(dom),
                     "launch_us": round(kus[dom], 2), "bytes_per_launch": b_dom,
                     "kernel_us": {k: round(v, 2) for k, v in kus.items()},
                     "timing": "HIP events on the solve stream around each launch, "
                               f"{rk['kernel_launches'][dom]} launches of a {CHECK * K}-iteration solve"},
    }

    # the mixed-precision form: FP32 products for the same K check periods
    sm = pdcs.settings_default(max_iter=CHECK * K, **FP32_ONLY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rm = prob.solve(sm)
    torch.cuda.synchronize()
    wall_m = time.perf_counter() - t0
    ips_m = rm["iterations"] / rm["solve_s"]
    kus_m, _ = kernel_timing(pdcs, prob, CHECK * K, **FP32_ONLY)
    log(f"mixed form: {ips_m:.1f} iter/s; kernels (us): "
        + ", ".join(f"{k} {v:.1f}" for k, v in kus_m.items()))
    out["mixed"] = {"form": "FP32 products (values and gathered x^, y^), FP64 iterates, "
                            "projections and checks, FP64 polish",
                    "iter_per_s": round(ips_m, 2), "ms_per_step": round(wall_m / K * 1e3, 3),
                    "speedup_iter_s": round(ips_m / ips, 3),
                    "kernel_us": {k: round(v, 2) for k, v in kus_m.items()}}
    # precision 2: the FP32 products plus FP32 lane-group SOC and exponential projections
    sp2 = pdcs.settings_default(max_iter=CHECK * K, **FP32_PROJ_ONLY)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rm2 = prob.solve(sp2)
    torch.cuda.synchronize()
    wall_m2 = time.perf_counter() - t0
    ips_m2 = rm2["iterations"] / rm2["solve_s"]
    kus_m2, _ = kernel_timing(pdcs, prob, CHECK * K, **FP32_PROJ_ONLY)
    log(f"mixed form with FP32 projections: {ips_m2:.1f} iter/s; kernels (us): "
        + ", ".join(f"{k} {v:.1f}" for k, v in kus_m2.items()))
    out["mixed_fp32_projections"] = {
        "form": "FP32 products and FP32 lane-group SOC / exponential projections (FP64 case tests "
                "and fallbacks), FP64 iterates and checks, FP64 polish (settings.precision 2)",
        "iter_per_s": round(ips_m2, 2), "ms_per_step": round(wall_m2 / K * 1e3, 3),
        "speedup_iter_s": round(ips_m2 / ips, 3),
        "kernel_us": {k: round(v, 2) for k, v in kus_m2.items()}}

    if not args.no_time_to_tol:
        def to_tol(**kw):
            t0 = time.perf_counter()
            rt = prob.solve(pdcs.settings_default(time_limit=100.0, **kw))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            rec = {"tol": 1e-6, "status": pdcs.SOLVE_STATUS[rt["status"]], "solve_s": round(rt["solve_s"], 3),
                   "setup_s": round(rt["setup_s"], 3), "wall_s": round(wall, 3),
                   "iterations": rt["iterations"], "restarts": rt["restarts"], "spmv": rt["spmv"],
                   "err_p": rt["err_p"], "err_d": rt["err_d"], "err_gap": rt["err_gap"],
                   "objective": rt["pobj"], "planted_objective": inst.opt,
                   "objective_rel_err": abs(rt["pobj"] - inst.opt) / max(1.0, abs(inst.opt))}
            log(f"time to 1e-6 {kw or ''}: {rt['solve_s']:.2f}s, {rt['iterations']} iterations, status "
                f"{pdcs.SOLVE_STATUS[rt['status']]}")
            return rt, rec
        rp_, out["time_to_tol"] = to_tol()
        xs = np.abs(rp_["x"]).max()
        for key, prec in (("mixed", 1), ("mixed_fp32_projections", 2)):
            rmx, rec = to_tol(precision=prec)
            rec["polish_iter"] = rmx["polish_iter"]
            rec["x_diff_vs_fp64_inf_rel"] = float(np.abs(rmx["x"] - rp_["x"]).max() / max(xs, 1e-300))
            rec["objective_diff_vs_fp64_rel"] = abs(rmx["pobj"] - rp_["pobj"]) / max(1.0, abs(rp_["pobj"]))
            out[key]["time_to_tol"] = rec
            out[key]["speedup_time_to_tol"] = round(rp_["solve_s"] / rmx["solve_s"], 3)

    if args.batch_count > 0:
        out["batched"] = batched_form(pdcs, instances, torch, args.batch_count)
    rec512 = batched_512_record()
    if rec512 is not None:
        out["batched_512_recorded"] = rec512
    if args.family_assets > 0:
        out["warm_start"] = warm_start_form(pdcs, instances, torch, args.family_assets,
                                            args.family_train, args.family_test)
    if not args.no_paper_workloads:
        extra = [tuple(int(v) for v in t.split("x")) for t in args.lasso_sizes.split(",") if t]
        out["paper_workloads"] = paper_workloads(pdcs, instances, torch, extra)
    if not args.no_projection_sweeps:
        out["projection_sweeps"] = projection_sweeps(pdcs, torch)
    if not args.no_ablation:
        out["pdhg_ablation"] = pdhg_ablation(pdcs, instances, torch)

    if not args.no_small:
        out["small_instance"] = small_instance(pdcs, instances, torch, not args.no_cpu_baseline)
    if not args.no_logistic:
        out["logistic"] = logistic_form(pdcs, instances, torch)

    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample ...")
        tt = out.get("time_to_tol", {})
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_iters,
                                           tt.get("iterations") if tt.get("status") == "optimal" else None)
        log(f"oracle: {out['cpu_baseline']['value']:.3f} iter/s on {out['cpu_baseline']['cores']} threads")

    prob.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

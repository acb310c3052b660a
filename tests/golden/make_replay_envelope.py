"""Writes replay_envelope.json: how far two correct FP64 runs of Algorithm 1
drift apart when they take the same decisions.

For each trajectory workload the oracle runs the default method (adaptive
step of Algorithm 1 line 4, adaptive reflection of line 5) for 200
iterations and logs its decisions.  A second build of the same oracle source,
compiled with FMA contraction (every a*b + c rounded once instead of twice),
then replays that decision log, and the relative iterate difference
||z_fma - z|| / max(1, ||z||) after every iteration is the envelope
(eta_envelope: the same for the step size used).  Both
runs are valid roundings of the same arithmetic, so no implementation can be
expected to stay closer to the oracle than this, up to a modest factor.
Calls only the oracle and the seeded generators:

    python tests/golden/make_replay_envelope.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2505_00311_amd import instances as I  # noqa: E402

ITERS = 200
WORKLOADS = {"small_mixed_0": lambda: I.small_mixed(0), "small_mixed_5": lambda: I.small_mixed(5),
             "lp_soc_n1000": lambda: I.lp_soc_small(20250501),
             "large_mixed_n20000": lambda: I.large_mixed(7, n=20000, m=10000)}


def rel_diffs(a, b):
    out = []
    for i in range(ITERS):
        za = np.concatenate([a["log"]["snap_x"][i], a["log"]["snap_y"][i]])
        zb = np.concatenate([b["log"]["snap_x"][i], b["log"]["snap_y"][i]])
        out.append(float(np.linalg.norm(zb - za) / max(1.0, np.linalg.norm(za))))
    return out


def main():
    oracle.build(force=False)
    fma = oracle.build_variant("fma", ["-ffp-contract=fast", "-mfma"])
    snaps = np.arange(1, ITERS + 1)
    res = {"cite": "Algorithm 1 (Section 3), default readings; iterates unscaled",
           "iterations": ITERS, "second_build": "gcc -O2 -ffp-contract=fast -mfma (FMA contraction)",
           "workloads": {}}
    for name, make in WORKLOADS.items():
        inst = make()
        s = oracle.default_settings(max_iter=ITERS)
        a = oracle.solve(inst, s, log_cap=ITERS, snap_iters=snaps)
        free = oracle.solve(inst, s, log_cap=ITERS, snap_iters=snaps, lib=fma)
        rep = oracle.solve(inst, s, log_cap=ITERS, snap_iters=snaps, lib=fma, replay=a["log"])
        diff = np.flatnonzero((a["log"]["attempts"] != free["log"]["attempts"]) |
                              (a["log"]["check_code"] != free["log"]["check_code"]))
        env = rel_diffs(a, rep)
        eta_env = np.abs(rep["log"]["eta_used"] / a["log"]["eta_used"] - 1.0)
        res["workloads"][name] = {
            "envelope": env,
            "eta_envelope": [float(v) for v in eta_env],
            "free_run_first_decision_difference": int(diff[0]) + 1 if diff.size else None,
            "oracle_margin_there": float(a["log"]["margin"][diff[0]]) if diff.size else None,
            "free_run_max": max(rel_diffs(a, free))}
        print(name, "envelope max", max(env), "at", int(np.argmax(env)) + 1, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "replay_envelope.json")
    with open(path, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()

"""Writes logistic_reference.json: the oracle's solution of the exponential-cone
logistic-regression workload (1e5 samples x 1e4 features, density 1e-3, seed
20250503) to max(err_p, err_d, err_gap) <= 1e-9, the reference objective that
the GPU forms' objective errors are measured against.  Calls only the oracle
and the seeded generator; the optional argument is the number of threads of
the oracle's timing mode (the reference then differs from a single-thread
run by rounding only):

    python tests/golden/make_logistic_reference.py [threads]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2505_00311_amd import instances as I  # noqa: E402

SEED, N, P, DENSITY, TOL = 20250503, 100_000, 10_000, 1e-3, 1e-9


def main():
    oracle.build(force=False)
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 1
    oracle.set_threads(threads)
    inst = I.logistic(SEED, samples=N, features=P, density=DENSITY)
    t0 = time.time()
    r = oracle.solve(inst, oracle.default_settings(tol=TOL, max_iter=10_000_000))
    wall = time.time() - t0
    x = r["x"]
    w = x[:P] - x[P:2 * P]
    out = dict(cite="configuration: sparse L1 logistic regression as an exponential-cone program "
                    "(exponential cone of Appendix A.2; termination measures of Section 5)",
               generator="instances.logistic", seed=SEED, samples=N, features=P, density=DENSITY,
               n=int(inst.n), m=int(inst.m), nnz=int(inst.nnz), tol=TOL,
               status=int(r["status"]), iterations=int(r["iterations"]),
               pobj=r["pobj"], dobj=r["dobj"], err_p=r["err_p"], err_d=r["err_d"],
               err_gap=r["err_gap"], oracle_wall_s=round(wall, 1), oracle_threads=threads,
               w_nonzeros=int(np.sum(np.abs(w) > 1e-9)),
               x_inf_norm=float(np.abs(x).max()), y_inf_norm=float(np.abs(r["y"]).max()))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "logistic_reference.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()

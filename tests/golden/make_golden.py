"""Write the oracle's reference results for the full-size workloads.

Runs oracle.ipm.solve (full-system FP64 IPM, CPU only) on the named workload
instances and stores the objective, iteration count, relative KKT score and
summary statistics of the solution as JSON next to this script.  Nothing here
touches the GPU path; the stored values are the oracle's.

Usage: python tests/golden/make_golden.py lowdof:100 fewEq:200 ...
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import ipm  # noqa: E402


def golden_path(workload: str, seed: int) -> str:
    return os.path.join(HERE, f"oracle_{workload}_{seed}.json")


def make(workload: str, seed: int) -> dict:
    qp = synth.workload(workload, seed=seed)
    t0 = time.perf_counter()
    r = ipm.solve(qp)
    dt = time.perf_counter() - t0
    out = dict(
        workload=workload, seed=seed, n=qp.n, m1=qp.m1, m2=qp.m2,
        obj=r.obj, iters=r.iters, rel_kkt=r.rel_kkt, converged=r.converged,
        x_norm2=float(np.linalg.norm(r.x)), x_sum=float(np.sum(r.x)),
        active=int(np.sum(r.nu > r.s)), seconds=dt,
        note="oracle.ipm.solve (full 4x4 Newton system, dense LU, FP64), tol 1e-10",
    )
    with open(golden_path(workload, seed), "w") as f:
        json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        w, s = arg.split(":")
        print(make(w, int(s)), flush=True)

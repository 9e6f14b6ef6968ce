"""Write the oracle's reference results for the full-size workloads.

Runs oracle.ipm.solve (full-system FP64 IPM, CPU only) on the named workload
instances and stores the objective, iteration count, relative KKT score and
summary statistics of the solution as JSON next to this script.  Nothing here
touches the GPU path; the stored values are the oracle's.

Usage: python tests/golden/make_golden.py lowdof:100 fewEq:200 set:batch24 set:large ...

  WORKLOAD:SEED  one instance of a named workload (synth.workload), one file
                 oracle_WORKLOAD_SEED.json
  set:batch24    the 24-QP sample synth.batch_sample() of the 512-QP batched draw
  set:large      synth.large_batch_sizes() (n = 1500, 2500, 4000)
                 one file oracle_set_NAME.json with a record per QP
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

SETS = {"batch24": synth.batch_sample, "large": synth.large_batch_sizes}


def golden_path(workload: str, seed: int) -> str:
    return os.path.join(HERE, f"oracle_{workload}_{seed}.json")


def set_path(name: str) -> str:
    return os.path.join(HERE, f"oracle_set_{name}.json")


def _record(qp, r, dt):
    return dict(
        n=qp.n, m1=qp.m1, m2=qp.m2, obj=r.obj, iters=r.iters, rel_kkt=r.rel_kkt, converged=r.converged,
        x_norm2=float(np.linalg.norm(r.x)), x_sum=float(np.sum(r.x)), active=int(np.sum(r.nu > r.s)), seconds=dt,
    )


def make(workload: str, seed: int) -> dict:
    qp = synth.workload(workload, seed=seed)
    t0 = time.perf_counter()
    r = ipm.solve(qp)
    dt = time.perf_counter() - t0
    out = dict(workload=workload, seed=seed, **_record(qp, r, dt),
               note="oracle.ipm.solve (full 4x4 Newton system, dense LU, FP64), tol 1e-10")
    with open(golden_path(workload, seed), "w") as f:
        json.dump(out, f, indent=1)
    return out


def _solve_spec(spec):
    from threadpoolctl import threadpool_limits
    seed, n, m1, m2 = spec
    qp = synth.gaussian_qp(seed, n, m1, m2)
    with threadpool_limits(1 if n <= 1100 else None):
        t0 = time.perf_counter()
        r = ipm.solve(qp)
        return dict(seed=seed, **_record(qp, r, time.perf_counter() - t0))


def make_set(name: str) -> dict:
    """Oracle solves of every gaussian_qp spec of the set (small ones in a process pool)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    specs = SETS[name]()
    small = [sp for sp in specs if sp[1] <= 1100]
    big = [sp for sp in specs if sp[1] > 1100]
    recs = {}
    if small:
        with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1), mp_context=mp.get_context("spawn")) as ex:
            for rec in ex.map(_solve_spec, small):
                recs[rec["seed"]] = rec
    for sp in big:
        recs[sp[0]] = _solve_spec(sp)
        print(f"  {name}: seed {sp[0]} n={sp[1]} done in {recs[sp[0]]['seconds']:.1f} s", flush=True)
    out = dict(set=name, records=[recs[sp[0]] for sp in specs],
               note="oracle.ipm.solve (full 4x4 Newton system, dense LU, FP64), tol 1e-10, on synth.gaussian_qp "
                    "(seed, n, m1, m2) of each record")
    with open(set_path(name), "w") as f:
        json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        w, s = arg.split(":")
        if w == "set":
            out = make_set(s)
            print(s, [(r["seed"], r["n"], r["iters"], r["converged"]) for r in out["records"]], flush=True)
        else:
            print(make(w, int(s)), flush=True)

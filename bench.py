"""Benchmark: QP solves per second of the implicit-PCG interior point method.

One step = one complete solve of a dense QP already resident in HBM: the K0
factorization (qp_factor_K0) and the interior point iteration with its
preconditioned CG solves (qp_ipm_solve).  Every solve is checked afterwards with
the oracle's relative KKT score (<= 1e-8) and, when the oracle's objective for
that instance is stored under tests/golden/, against it (1e-7 relative); only
passing solves count.

Prints one JSON line.  Extra objects:
  roofline      the dominant CG-step kernel: algorithmic bytes per launch over
                its average launch time, sampled with HIP events on the
                library's stream during the timed solves (qp_profile_get);
                traffic from the committed rocprofv3 counter summary when it was
                taken on the current kernel source, else null
  cpu_baseline  the oracle on this host's cores, a bounded sample of the same
                instance extrapolated to a whole solve
Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload lowdof]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QP solves/s at rel KKT res 1e-8 (batched FP32 vs plain FP64); HBM GB/s; p99 lat"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "lowdof": dict(desc="one dense QP n=4096, m1=3072 equalities, m2=2048 inequalities, low-dof P_L",
                   prec="PL", seeds=[100, 101, 102]),
    "fewEq": dict(desc="one dense QP n=4096, m1=256, m2=4096, H eigenvalues 1e-4..1e2, few-equalities P_H",
                  prec="PH", seeds=[200, 201, 202]),
    "small": dict(desc="one dense QP n=200, m1=50, m2=100", prec="PH", seeds=list(range(16))),
}
OP_NAMES = ["gemv_cols_part_kernel<T,1> (C^T p)", "gemv_rows_kernel<T,2> (Sigma M u)",
            "gemv_cols_part_kernel<T,3> (M^T v)", "pcg_q_kernel<T> (C w + D p)",
            "gemv_rows_kernel<T,4> (X_P r)", "gemv_cols_part_kernel<T,5> (X_P^T t)"]


def op_bytes(n, m1, m2, elem):
    """Algorithmic matrix bytes per launch of each CG-step sweep."""
    m_entries = n * (n + 1) // 2 + m1 * n          # M = L^{-1}[:, :n], lower trapezoid
    xp_entries = m2 * (m2 + 1) // 2                # X_P, lower triangle
    return [m2 * n * elem, m_entries * elem, m_entries * elem, m2 * n * elem, xp_entries * elem, xp_entries * elem]


def kernel_src_hash():
    h = hashlib.sha256()
    for f in ("gemv.hip", "gemv_core.hpp", "pcg.hip", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2104_12916_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, kernel_tag):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, "no counter summary committed"
    with open(path) as f:
        t = json.load(f)
    rec = t.get(f"{workload}:{kernel_tag}")
    if rec is None:
        return None, "no counters for this kernel/workload"
    if rec.get("src_hash") != kernel_src_hash():
        return None, "kernel source changed since the counters were taken"
    return rec["bytes_per_launch"], rec.get("note", "")


def golden(workload, seed):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}_{seed}.json")
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return None


def cpu_baseline(workload, seed, sample_iters, gpu_iters):
    """Time the oracle on a bounded sample of the same instance and extrapolate."""
    import synth
    from oracle import ipm
    from threadpoolctl import threadpool_info
    qp = synth.workload(workload, seed=seed)
    t0 = time.perf_counter()
    ipm.validate(qp)
    ti = time.perf_counter()
    ipm.initial_point(qp)
    t1 = time.perf_counter()
    r = ipm.solve(qp, check=False, max_iters_cap=sample_iters)
    t2 = time.perf_counter()
    # the capped run computes the initial point again; take it out of the per-iteration time
    per_iter = max(1e-9, (t2 - t1) - (t1 - ti)) / max(1, r.iters)
    g = golden(workload, seed)
    if g is not None:
        n_it, src = g["iters"], "oracle iteration count from tests/golden"
    else:
        n_it, src = gpu_iters, "iteration count of the GPU solve of the same instance"
    est = (t1 - t0) + n_it * per_iter
    threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
    return {
        "value": 1.0 / est, "unit": "QP solves/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"seed {seed}: validation + initial point ({t1 - t0:.2f} s) and {r.iters} full-system IPM "
                   f"iterations ({per_iter:.2f} s each, dense LU of the {qp.n + qp.m1 + 2 * qp.m2}-square Newton "
                   f"matrix), extrapolated to {n_it} iterations ({src}); {os.cpu_count()} host CPUs"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lowdof", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["PL", "PH", "none", "auto"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (independent QPs shard "
              "across GPUs with no exchange, and this build measures one GPU's share).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from oracle import kkt
    from paper_2104_12916_amd import qpgpu

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    prec_name = args.prec or w["prec"]
    prec = {"PL": qpgpu.QP_PREC_LOW_DOF, "PH": qpgpu.QP_PREC_FEW_EQ, "none": qpgpu.QP_PREC_NONE,
            "auto": qpgpu.QP_PREC_AUTO}[prec_name]
    precision = qpgpu.QP_MIXED if args.precision == "mixed" else qpgpu.QP_FP64
    seeds = w["seeds"][:max(1, min(len(w["seeds"]), args.steps))]
    qps, solvers = [], []
    for sd in seeds:
        qp = synth.workload(args.workload, seed=sd)
        qps.append(qp)
        solvers.append(qpgpu.Solver(*qp.arrays(), prec=prec, precision=precision, profile=1))
    torch.cuda.synchronize()

    def step(i):
        s = solvers[i % len(solvers)]
        s.factor()
        x, lam, nu, sl, info = s.ipm(accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))
        return i % len(solvers), x, lam, nu, info

    for i in range(args.warmup):
        step(i)
        print(f"warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    for s in solvers:
        s.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for i in range(args.steps):
        outs.append(step(i))
        print(f"step {i + 1}/{args.steps}: ipm {outs[-1][4].ipm_iters} it, cg {outs[-1][4].pcg_iters_total}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0

    # parity of every timed solve (oracle's KKT score on the host; objective vs stored oracle value)
    ok = 0
    worst_kkt, worst_obj = 0.0, 0.0
    ipm_iters, cg_iters = [], []
    for k, x, lam, nu, info in outs:
        qp = qps[k]
        sc, _ = kkt.rel_kkt(qp, x, lam, nu)
        f = kkt.objective(qp, x)
        g = golden(args.workload, seeds[k])
        oerr = abs(f - g["obj"]) / max(1.0, abs(g["obj"])) if g else 0.0
        worst_kkt, worst_obj = max(worst_kkt, sc), max(worst_obj, oerr)
        if sc <= 1e-8 and oerr <= 1e-7:
            ok += 1
        ipm_iters.append(info.ipm_iters)
        cg_iters.append(info.pcg_iters_total)

    # dominant kernel from the sampled launch times of the timed solves
    ms = np.zeros(6)
    cnt = np.zeros(6)
    for s in solvers:
        m, c = s.profile()
        ms += np.array(m) * np.array(c)
        cnt += np.array(c)
    avg_ms = np.divide(ms, cnt, out=np.zeros(6), where=cnt > 0)
    qp0 = qps[0]
    elem = 4 if precision == qpgpu.QP_MIXED else 8
    nbytes = op_bytes(qp0.n, qp0.m1, qp0.m2, elem)
    ops = {}
    for o in range(6):
        if cnt[o] > 0:
            ops[OP_NAMES[o]] = dict(avg_us=round(avg_ms[o] * 1e3, 2), samples=int(cnt[o]),
                                    bytes=nbytes[o], gbs=round(nbytes[o] / (avg_ms[o] * 1e-3) / 1e9, 1))
    dom = int(np.argmax(avg_ms))
    achieved = nbytes[dom] / (avg_ms[dom] * 1e-3) / 1e9
    traffic, tnote = load_traffic(args.workload, ["C^T", "M", "M^T", "q", "XP", "XP^T"][dom])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=OP_NAMES[dom],
                    bytes_per_launch=nbytes[dom], avg_launch_us=round(avg_ms[dom] * 1e3, 2),
                    traffic_note=tnote)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, seeds[0], args.cpu_sample_iters, ipm_iters[0])

    value = ok / elapsed
    line = {
        "metric": METRIC, "value": value, "unit": "QP solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if precision == qpgpu.QP_MIXED else "f64",
        "data": "synthetic (seeded dense Gaussian QPs resident in HBM)",
        "config": {"workload": f"{args.workload}: {w['desc']}", "seeds": seeds, "precond": prec_name,
                   "precision": args.precision},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": dict(passed=ok, solves=len(outs), max_rel_kkt=worst_kkt, max_obj_rel_err=worst_obj),
        "ipm_iters": ipm_iters, "cg_iters": cg_iters,
        "us_per_cg_step": round(elapsed / max(1, sum(cg_iters)) * 1e6, 2),
        "cg_step_sweeps": ops,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: QP solves per second of the implicit-PCG interior point method.

One step = one complete solve of a dense QP already resident in HBM: the K0
factorization (qp_factor_K0) and the interior point iteration with its
preconditioned CG solves (qp_ipm_solve).  Every solve is checked afterwards:
the relative KKT score the library reports for the returned iterate (computed
in float64 on the GPU; tests/ pin it to the oracle's score of the same
iterate) must be <= 1e-8 and, when the oracle's objective for that instance is
stored under tests/golden/, the objective must match it (1e-7 relative); only
passing solves count.  The oracle itself runs only in the cpu_baseline leg.

Prints one JSON line.  Extra objects:
  roofline      the dominant CG-step kernel: algorithmic bytes per launch over
                its average launch time, sampled with HIP events on the
                library's stream during the timed solves (qp_profile_get);
                traffic from the committed rocprofv3 counter summary when it was
                taken on the current kernel source, else null
  cpu_baseline  the oracle on this host's cores: one whole timed solve of the
                same instance (the full-system IPM to its own tolerance)
  batch         the 512-QP batched workload beside the headline: batched mixed
                precision, batched float64 and the single-QP float64 path over
                the same QPs resident in HBM (solves/s each), the share of CG
                steps run in float64, and the objectives of a fixed 24-QP sample
                against the oracle's stored values (tests/golden)
  cg_per_ipm_iter  CG steps of every predictor and corrector solve of one
                headline solve beside the Theorem thm1 / thm2 bound
Usage: python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload lowdof]

--workload batch: 512 independent QPs (n ~ U{64..1024}, m1 = n/4, m2 = n/2)
  solved together through qp_batch_*, inputs resident in HBM; a step is the
  whole batch.  Also times the single-QP float64 path over the same QPs.
--workload serve: a stream of QPs of log-uniform size arriving from host
  memory; saturated throughput, then Poisson arrivals at 0.5x and 0.8x of it
  with p50/p99 latency from arrival to result.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QP solves/s at rel KKT res 1e-8 (batched FP32 vs plain FP64); HBM GB/s; p99 lat"
HBM_PEAK_GBS = 8000.0

BATCH_DESC = ("512 independent dense QPs, n ~ U{64..1024}, m1 = n/4, m2 = n/2 (seeds 1000+i), "
              "preconditioner by the smaller CG bound (P_H here), batched in one qp_batch")
SERVE_DESC = ("stream of dense QPs, n log-uniform 128..4096, m1 = n U(1/8, 1/2), m2 = n U(1/2, 1) "
              "(stream seed 5000, request i seed 1e6+i), continuous batching under a memory budget")
WORKLOADS = {
    "lowdof": dict(desc="one dense QP n=4096, m1=3072 equalities, m2=2048 inequalities, low-dof P_L",
                   prec="PL", seeds=[100, 101, 102]),
    "fewEq": dict(desc="one dense QP n=4096, m1=256, m2=4096, H eigenvalues 1e-4..1e2, few-equalities P_H",
                  prec="PH", seeds=[200, 201, 202]),
    "small": dict(desc="one dense QP n=200, m1=50, m2=100", prec="PH", seeds=list(range(16))),
    "batch": dict(desc=BATCH_DESC, prec="auto", seeds=[1000]),
    "serve": dict(desc=SERVE_DESC, prec="auto", seeds=[5000]),
    "shared": dict(desc="k dense QPs sharing H, A, C of the low-dof instance (n=4096, m1=3072, m2=2048, seed 100) "
                        "with their own c, b, d (synth.shared_family), P_L, one K0 factorization, block PCG",
                   prec="PL", seeds=[100]),
}
OP_NAMES = ["gemv_rows_kernel<T,1> (C^T p over stored C^T)", "gemv_rows_kernel<T,2> (Sigma M u)",
            "gemv_rows_kernel<T,3> (M^T v over stored M^T)", "pcg_q_kernel<T> (C w + D p)",
            "gemv_rows_kernel<T,4> (X_P r)", "gemv_cols_part_kernel<T,5> (X_P^T t)"]
# with the one-pass K0 product, slots 1 and 2 hold its sweep and the sum of its partials, and
# slots 4 and 5 the one-pass P_H apply X_P^T X_P r (m2 <= 4096) and the sum of its partials
# (in the folded CG step, the default for P_H and for the n <= 4096 size bucket, slot 0 is
# fold_ct_kernel, slot 2 k0_sym_reduce_fold_kernel, slot 3 fold_q_kernel and slot 5
# ph_reduce_fold_kernel: the same matrices with the vector update folded in)
OP_NAMES_ONE_PASS = ["gemv_rows_kernel<T,1> / fold_ct_kernel<T> (C^T p over stored C^T)",
                     "k0_sym_kernel<T> (M^T Sigma M u, one pass over M)",
                     "k0_sym_reduce[_fold]_kernel<T> (sum of the per-workgroup partials of w)",
                     "pcg_q_kernel<T> / fold_q_kernel<T> (C w + D p)",
                     "k0_sym_kernel<T> over X_P (X_P^T X_P r, one pass)",
                     "k0_sym_reduce_kernel<T> / ph_reduce_fold_kernel<T> (sum of the partials of z)"]
ONE_PASS_MAX = 4096  # widest operand of the float64 one-pass sweep


def op_bytes(n, m1, m2, elem):
    """Algorithmic matrix bytes per launch of each CG-step sweep."""
    m_entries = n * (n + 1) // 2 + m1 * n          # M = L^{-1}[:, :n], lower trapezoid
    xp_entries = m2 * (m2 + 1) // 2                # X_P, lower triangle
    return [m2 * n * elem, m_entries * elem, m_entries * elem, m2 * n * elem, xp_entries * elem, xp_entries * elem]


def load_traffic(workload, kernel_tag):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, "no counter summary committed"
    with open(path) as f:
        t = json.load(f)
    rec = t.get(f"{workload}:{kernel_tag}")
    if rec is None:
        return None, "no counters for this kernel/workload"
    from paper_2104_12916_amd.profile_summary import kernel_src_hash
    if rec.get("src_hash") != kernel_src_hash():
        return None, "kernel source changed since the counters were taken"
    return rec["bytes_per_launch"], rec.get("note", "")


def golden(workload, seed):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}_{seed}.json")
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return None


def golden_set(name):
    """Stored oracle results of a named instance set ({seed: record}; {} if absent)."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_set_{name}.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return {r["seed"]: r for r in json.load(f)["records"]}


def cpu_baseline_full(workload, seed):
    """One whole oracle solve of the same instance, timed on this host's cores."""
    import synth
    from oracle import ipm
    from threadpoolctl import threadpool_info
    qp = synth.workload(workload, seed=seed)
    t0 = time.perf_counter()
    r = ipm.solve(qp)
    el = time.perf_counter() - t0
    threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
    return {
        "value": 1.0 / el, "unit": "QP solves/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"one whole solve of seed {seed}: validation, initial point and {r.iters} full-system IPM "
                   f"iterations (dense LU of the {qp.n + qp.m1 + 2 * qp.m2}-square Newton matrix) to rel KKT "
                   f"{r.rel_kkt:.1e} in {el:.1f} s; {os.cpu_count()} host CPUs"),
    }


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


def _oracle_solve_timed(spec):
    """Worker of the CPU baseline pool: one oracle solve with one BLAS thread."""
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import ipm
    seed, n, m1, m2 = spec
    qp = synth.gaussian_qp(seed, n, m1, m2)
    with threadpool_limits(1):
        t = time.perf_counter()
        ipm.solve(qp)
        return time.perf_counter() - t


def cpu_baseline_pool(specs, budget_s=20.0):
    """Oracle throughput on independent QPs: one process per host core, one BLAS
    thread each, over a bounded sample of the workload's instances."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    workers = min(16, os.cpu_count() or 1)
    times = []
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(_oracle_solve_timed, sp) for sp in specs]
        for f in futs:
            times.append(f.result())
            if time.perf_counter() - t0 > budget_s:
                for g in futs:
                    g.cancel()
                break
    done = len(times)
    rate = workers * done / max(1e-9, sum(times))
    return {"value": rate, "unit": "QP solves/s", "cores": workers, "kind": "oracle",
            "sample": (f"{done} instances of the workload (n = {min(s[1] for s in specs[:done])}.."
                       f"{max(s[1] for s in specs[:done])}), full-system oracle IPM, {workers} processes x 1 BLAS thread; "
                       f"rate = processes x solves / summed solve time (generation excluded)")}


def batch_roofline(prof, elem):
    """Dominant batched sweep: algorithmic bytes per sampled launch over its time."""
    ms, by, cnt = prof
    names = ["bgemv_rows_kernel<T,1> (C^T p over stored C^T)", "bgemv_rows_kernel<T,2> (Sigma M u)",
             "bgemv_rows_kernel<T,3> (M^T v over stored M^T)", "bpcg_q_kernel<T> (C w + D p)",
             "bgemv_rows_kernel<T,4> (X_P r)", "bgemv_cols_part_kernel<T,5> (X_P^T t)"]
    if cnt[1] > 0 and by[2] == 0:  # one pass over M: slot 1 is that sweep (its partial sums carry no matrix bytes)
        names[1] = "bk0_sym_kernel<T> (M^T Sigma M u, one pass over M)"
        names[2] = "bk0_sym_reduce_kernel<T> (sum of the partials of w)"
    if cnt[4] > 0 and by[5] == 0:  # one pass over X_P in the P_H apply, then the sum of its partials
        names[4] = "bk0_sym_kernel<T> over X_P (X_P^T X_P r, one pass)"
        names[5] = "bk0_sym_reduce_kernel<T> (sum of the partials of z)"
    ops = {}
    for o in range(6):
        if cnt[o] > 0 and ms[o] > 0:
            ops[names[o]] = dict(avg_us=round(ms[o] * 1e3, 2), samples=int(cnt[o]), avg_bytes=int(by[o]),
                                 gbs=round(by[o] / (ms[o] * 1e-3) / 1e9, 1))
    if not ops:
        return None, ops
    dom = max(range(6), key=lambda o: ms[o] if cnt[o] else -1)
    ach = by[dom] / (ms[dom] * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4),
                traffic=None, kernel=names[dom], bytes_per_launch=int(by[dom]), avg_launch_us=round(ms[dom] * 1e3, 2),
                traffic_note="no counters taken for the batched sweeps"), ops


def batch_instances(count):
    """The batched workload's QPs, generated on the host and copied to HBM once."""
    import torch
    import synth
    sizes = synth.batch_sizes(count, 1000)
    t = time.perf_counter()
    qps = [synth.gaussian_qp(*sz) for sz in sizes]
    print(f"generated {len(qps)} QPs in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    dev = [tuple(torch.from_numpy(a).cuda() for a in qp.arrays()) for qp in qps]
    torch.cuda.synchronize()
    return sizes, qps, dev


def solve_batch(dev, k, budget, profile=False, **opts):
    """Admit the first k resident QPs into one batch and run it to the end.
    Returns (seconds, [(x, lam, nu, s, info)], ticks, sampled profile)."""
    import torch
    from paper_2104_12916_amd import qpgpu
    b = qpgpu.Batch(budget, profile=int(profile), **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [b.admit(*dev[i]) for i in range(k)]
    assert all(tk is not None for tk in tickets), "batch budget too small"
    rounds = 0
    while b.query()["in_flight"]:
        b.step(1)
        rounds += 1
    out = [b.collect(tk, accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV)) for tk in tickets]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = b.profile() if profile else None
    b.close()
    return el, out, rounds, prof


def batch_quality(sizes, res, gold):
    """Parity and work counts of one batched run: every QP's reported KKT score,
    the objectives of the stored oracle sample, CG steps and their float64 share."""
    from paper_2104_12916_amd import qpgpu
    bad, worst, worst_obj, sampled = set(), 0.0, 0.0, 0
    ipm_it, cg, cg64, fb = [], 0, 0, 0
    for i, (x, lam, nu, s, info) in enumerate(res):
        worst = max(worst, info.rel_kkt)
        ok = info.rel_kkt <= 1e-8 and info.status == qpgpu.QP_OK
        g = gold.get(sizes[i][0])
        if g is not None:
            e = abs(info.obj - g["obj"]) / max(1.0, abs(g["obj"]))
            worst_obj = max(worst_obj, e)
            sampled += 1
            ok = ok and e <= 1e-7
        if not ok:
            bad.add(i)
        ipm_it.append(info.ipm_iters)
        cg += info.pcg_iters_total
        cg64 += info.pcg_iters_fp64
        fb += info.fp64_fallbacks
    return dict(passed=len(res) - len(bad), solves=len(res), max_rel_kkt=worst,
                sample_max_obj_rel_err=worst_obj, sample_checked=sampled,
                ipm_iters_range=[min(ipm_it), max(ipm_it)], reduced_solves=2 * sum(ipm_it),
                fp64_fallback_solves=fb, cg_steps=int(cg), cg_steps_fp64=int(cg64),
                fp64_cg_share=round(cg64 / max(1, cg), 4))


def single_qp_loop(dev, qps, k, prec):
    """The plain single-QP float64 path over the first k resident QPs, one after another."""
    import torch
    from paper_2104_12916_amd import qpgpu
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(k):
        sv = qpgpu.Solver(*dev[i], prec=prec)
        sv.factor()
        x = torch.empty(qps[i].n, dtype=torch.float64, device="cuda")
        lam = torch.empty(qps[i].m1, dtype=torch.float64, device="cuda")
        nu = torch.empty(qps[i].m2, dtype=torch.float64, device="cuda")
        sl = torch.empty(qps[i].m2, dtype=torch.float64, device="cuda")
        st_, info = qpgpu.qp_ipm_solve(sv.ctx, x, lam, nu, sl)
        infos.append(info)
        sv.close()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, infos


def config4_legs(count=512, single=True):
    """The 512-QP batched workload: batched mixed, batched float64 and the single-QP
    float64 loop over the same QPs in HBM (factorization and every IPM iteration inside
    the clock; one 16-QP warm-up batch per precision first)."""
    from paper_2104_12916_amd import qpgpu
    sizes, qps, dev = batch_instances(count)
    gold = golden_set("batch24")
    out = {"workload": BATCH_DESC, "qps": count}
    for name, precision in (("batched_mixed", qpgpu.QP_MIXED), ("batched_fp64", qpgpu.QP_FP64)):
        opt = qpgpu.qp_default_options(prec=qpgpu.QP_PREC_AUTO, precision=precision)
        budget = int(1.05 * sum(qpgpu.qp_batch_footprint(opt, q.n, q.m1, q.m2) for q in qps)) + (64 << 20)
        solve_batch(dev, min(16, count), budget, prec=qpgpu.QP_PREC_AUTO, precision=precision)
        el, res, rounds, _ = solve_batch(dev, count, budget, prec=qpgpu.QP_PREC_AUTO, precision=precision)
        q = batch_quality(sizes, res, gold)
        out[name] = dict(value=round(q["passed"] / el, 2), unit="QP solves/s", seconds=round(el, 3), ticks=rounds,
                         dtype="f32+f64" if precision == qpgpu.QP_MIXED else "f64", **q)
        print(f"config-4 {name}: {count} QPs in {el:.2f} s, {q['passed']} pass, fp64 CG share "
              f"{q['fp64_cg_share']}", file=sys.stderr, flush=True)
    if single:
        el, infos = single_qp_loop(dev, qps, count, qpgpu.QP_PREC_AUTO)
        res = [(None, None, None, None, i) for i in infos]
        q = batch_quality(sizes, res, gold)
        out["single_qp_fp64"] = dict(value=round(q["passed"] / el, 2), unit="QP solves/s", seconds=round(el, 3),
                                     path="qp_setup + qp_factor_K0 + qp_ipm_solve per QP, float64", **q)
        print(f"config-4 single-QP fp64 loop: {count} QPs in {el:.2f} s", file=sys.stderr, flush=True)
        base = out["single_qp_fp64"]["value"]
        out["speedup_batched_mixed_vs_single_fp64"] = round(out["batched_mixed"]["value"] / base, 2)
        out["speedup_batched_fp64_vs_single_fp64"] = round(out["batched_fp64"]["value"] / base, 2)
    out["speedup_mixed_vs_fp64_batched"] = round(out["batched_mixed"]["value"] / out["batched_fp64"]["value"], 3)
    return out


def run_batch_workload(args):
    import numpy as np
    import torch
    import synth
    from paper_2104_12916_amd import qpgpu
    torch.cuda.set_device(0)
    prec = {"PL": qpgpu.QP_PREC_LOW_DOF, "PH": qpgpu.QP_PREC_FEW_EQ, "none": qpgpu.QP_PREC_NONE,
            "auto": qpgpu.QP_PREC_AUTO}[args.prec or "auto"]
    precision = qpgpu.QP_FP64 if args.precision == "fp64" else qpgpu.QP_MIXED
    kf = qpgpu.QP_KF_EXPLICIT if args.kf == "explicit" else qpgpu.QP_KF_IMPLICIT
    sizes, qps, dev = batch_instances(args.batch_count)
    opt = qpgpu.qp_default_options(prec=prec, precision=precision, kf_form=kf)
    budget = int(1.05 * sum(qpgpu.qp_batch_footprint(opt, q.n, q.m1, q.m2) for q in qps)) + (64 << 20)

    def solve_all(k, profile):
        return solve_batch(dev, k, budget, profile, prec=prec, precision=precision, kf_form=kf)

    for w in range(args.warmup):
        solve_all(min(16, len(qps)), False)
        print(f"warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    steps = max(1, args.steps)
    times, res, prof = [], None, None
    for st in range(steps):
        el, out, rounds, p = solve_all(len(qps), st == 0)
        times.append(el)
        if st == 0:
            res, prof = out, p
        print(f"step {st + 1}/{steps}: {len(qps)} QPs in {el:.2f} s ({rounds} rounds)", file=sys.stderr, flush=True)
    elapsed = sum(times)
    # every result's reported KKT score, and the stored oracle objectives of the 24-QP sample
    quality = batch_quality(sizes, res, golden_set("batch24"))
    ok, worst = quality["passed"], quality["max_rel_kkt"]
    print(f"parity: {ok}/{len(qps)} pass; worst rel_kkt {worst:.2e}", file=sys.stderr, flush=True)
    # the single-QP float64 path over the same resident QPs
    single = None
    if args.single_count > 0:
        k = min(args.single_count, len(qps))
        el, _ = single_qp_loop(dev, qps, k, prec)
        single = dict(value=k / el, unit="QP solves/s", qps=k, seconds=round(el, 3),
                      path="qp_setup + qp_factor_K0 + qp_ipm_solve per QP, float64, inputs in HBM")
        print(f"single-QP fp64 loop: {k} QPs in {el:.2f} s", file=sys.stderr, flush=True)
    elem = 4 if precision == qpgpu.QP_MIXED else 8
    roof, ops = batch_roofline(prof, elem)
    cpu = None
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(0)
        pick = sorted(rng.choice(len(sizes), size=min(48, len(sizes)), replace=False))
        cpu = cpu_baseline_pool([sizes[i] for i in pick])
    value = ok * steps / elapsed
    line = {
        "metric": METRIC, "value": value, "unit": "QP solves/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if precision == qpgpu.QP_MIXED else "f64",
        "data": "synthetic (seeded dense Gaussian QPs resident in HBM)",
        "config": {"workload": f"batch: {BATCH_DESC}", "qps": len(qps), "precond": args.prec or "auto",
                   "precision": args.precision, "kf_form": args.kf, "budget_bytes": budget},
        "roofline": roof, "cpu_baseline": cpu,
        "parity": dict(note="rel KKT score the library reports per QP; objectives of the 24-QP sample against "
                            "the oracle's stored values", **quality),
        "single_qp_fp64_gpu": single,
        "speedup_vs_single_qp_fp64": (value / single["value"]) if single else None,
        "batched_sweeps": ops,
    }
    print(json.dumps(line), flush=True)


def run_shared_workload(args):
    """k QPs that share H, A, C: one factorization, block PCG, lockstep IPMs (qp_shared_*)."""
    import numpy as np
    import torch
    import synth
    from paper_2104_12916_amd import qpgpu

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    k = args.shared_k
    base = synth.workload("lowdof", seed=100)
    fam = synth.shared_family(100, base.n, base.m1, base.m2, k, base=base)
    cs, bs, ds = (np.stack([getattr(q, f) for q in fam]) for f in ("c", "b", "d"))
    print(f"shared: {k} QPs n={base.n} m1={base.m1} m2={base.m2}", file=sys.stderr, flush=True)

    def solve():
        t0 = time.perf_counter()
        sh = qpgpu.Shared(base.H, base.A, base.C, prec=qpgpu.QP_PREC_LOW_DOF)  # factorization inside the clock
        out = sh.ipm(cs, bs, ds)
        torch.cuda.synchronize()
        sh.close()
        return time.perf_counter() - t0, out

    for _ in range(args.warmup):
        solve()
    times, out = [], None
    for i in range(args.steps):
        dt, out = solve()
        times.append(dt)
        print(f"step {i + 1}/{args.steps}: {k} QPs in {dt:.2f} s", file=sys.stderr, flush=True)
    x, lam, nu, s, infos = out
    worst, ok = 0.0, 0
    for j in range(k):
        sc = infos[j].rel_kkt  # reported score of QP j (pinned to the oracle's in tests/test_gpu_shared.py)
        worst = max(worst, sc)
        ok += sc <= 1e-8
    # the same QPs one at a time through the single-QP path (factorization each time), for comparison
    single = None
    if args.single_count > 0:
        m = min(args.single_count, k)
        t0 = time.perf_counter()
        for q in fam[:m]:
            sv = qpgpu.Solver(*q.arrays(), prec=qpgpu.QP_PREC_LOW_DOF)
            sv.factor()
            sv.ipm()
            sv.close()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        single = dict(value=m / el, unit="QP solves/s", qps=m, seconds=round(el, 2))
    elapsed = sum(times)
    value = k * args.steps / elapsed
    line = {
        "metric": METRIC, "value": value, "unit": "QP solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded dense Gaussian QPs resident in HBM)",
        "config": {"workload": "shared: " + WORKLOADS["shared"]["desc"], "qps": k, "precond": "PL",
                   "precision": "fp64", "kf_form": "implicit"},
        "roofline": None, "cpu_baseline": None,
        "parity": dict(passed=ok, solves=k, max_rel_kkt=worst),
        "ipm_iters": [i.ipm_iters for i in infos], "cg_steps": [int(i.pcg_iters_total) for i in infos],
        "single_qp_fp64_gpu": single,
        "speedup_vs_single_qp_fp64": (value / single["value"]) if single else None,
    }
    print(json.dumps(line), flush=True)


def run_serve_workload(args):
    import collections
    import numpy as np
    import torch
    import synth
    from paper_2104_12916_amd import qpgpu
    torch.cuda.set_device(0)
    prec = {"PL": qpgpu.QP_PREC_LOW_DOF, "PH": qpgpu.QP_PREC_FEW_EQ, "none": qpgpu.QP_PREC_NONE,
            "auto": qpgpu.QP_PREC_AUTO}[args.prec or "auto"]
    precision = qpgpu.QP_FP64 if args.precision == "fp64" else qpgpu.QP_MIXED
    kf = qpgpu.QP_KF_EXPLICIT if args.kf == "explicit" else qpgpu.QP_KF_IMPLICIT
    nw, nm = args.serve_warmup, args.serve_requests
    specs = synth.serving_stream(nw + nm, seed=5000)
    t = time.perf_counter()
    reqs = []
    for sp in specs:
        reqs.append(synth.gaussian_qp(*sp))
        if len(reqs) % 250 == 0:
            print(f"  generated {len(reqs)}/{len(specs)}", file=sys.stderr, flush=True)
    print(f"generated {len(reqs)} requests in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    budget = int(args.serve_budget_gb * (1 << 30))

    def serve(rate):
        """Run the stream; rate None admits everything at t = 0 (saturation)."""
        rng = np.random.default_rng(5001)
        gaps = np.zeros(len(reqs)) if rate is None else rng.exponential(1.0 / rate, size=len(reqs))
        arrive = np.cumsum(gaps)
        b = qpgpu.Batch(budget, prec=prec, precision=precision, kf_form=kf)
        pending = collections.deque()
        owner, lat, results = {}, {}, {}
        t0 = time.perf_counter()
        i = done = 0
        while done < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and arrive[i] <= now:
                pending.append(i)
                i += 1
            while pending:
                tk = b.admit(*reqs[pending[0]].arrays())
                if tk is None:
                    break
                owner[tk] = pending.popleft()
            if b.query()["in_flight"]:
                b.step(1)
            elif i < len(reqs):
                time.sleep(max(0.0, arrive[i] - (time.perf_counter() - t0)))
            for tk in b.finished():
                k = owner.pop(tk)
                results[k] = b.collect(tk, accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))
                lat[k] = time.perf_counter() - t0 - arrive[k]
                done += 1
                if done % 250 == 0:
                    print(f"  {done}/{len(reqs)} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        b.close()
        meas = list(range(nw, len(reqs)))
        t_first = min(arrive[k] for k in meas)
        t_last = max(arrive[k] + lat[k] for k in meas)
        lm = np.array([lat[k] for k in meas]) * 1e3
        return results, dict(solves_per_s=len(meas) / max(1e-9, t_last - t_first), p50_ms=float(np.percentile(lm, 50)),
                             p99_ms=float(np.percentile(lm, 99)), mean_ms=float(lm.mean()))

    res_sat, sat = serve(None)
    x_rate = sat["solves_per_s"]
    print(f"saturated: {x_rate:.2f} solves/s", file=sys.stderr, flush=True)
    loads = {}
    for f in (0.5, 0.8):
        _, st_ = serve(f * x_rate)
        loads[f"{f}X"] = {k: round(v, 3) for k, v in st_.items()}
        print(f"load {f}X: {st_}", file=sys.stderr, flush=True)
    ok, worst = 0, 0.0
    for k in range(nw, len(reqs)):
        x, lam, nu, s, info = res_sat[k]
        worst = max(worst, info.rel_kkt)  # the reported score of the returned iterate
        ok += int(info.rel_kkt <= 1e-8 and info.status == qpgpu.QP_OK)
    # alone-versus-mix equality on the smallest requests
    small = sorted(range(nw, len(reqs)), key=lambda k: reqs[k].n)[:3]
    same = True
    for k in small:
        b = qpgpu.Batch(budget, prec=prec, precision=precision, kf_form=kf)
        tk = b.admit(*reqs[k].arrays())
        b.step(10 ** 6)
        xa = b.collect(tk, accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))[0]
        b.close()
        same = same and bool(np.array_equal(xa, res_sat[k][0]))
    line = {
        "metric": METRIC, "value": x_rate * ok / nm, "unit": "QP solves/s", "n_gpus": 1, "steps": nm,
        "warmup": nw, "ms_per_step": 1e3 / max(1e-9, x_rate), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if precision == qpgpu.QP_MIXED else "f64",
        "data": "synthetic (seeded dense Gaussian QPs arriving from host memory; admission includes the upload)",
        "config": {"workload": f"serve: {SERVE_DESC}", "requests": nm, "warmup_requests": nw,
                   "budget_gb": args.serve_budget_gb, "precond": args.prec or "auto", "precision": args.precision,
                   "kf_form": args.kf},
        "latency": {"saturated": {k: round(v, 3) for k, v in sat.items()}, **loads},
        "parity": dict(passed=ok, solves=nm, max_rel_kkt=worst, alone_equals_mix=same, checked_alone=len(small)),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lowdof", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["PL", "PH", "none", "auto"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--kf", default="implicit", choices=["implicit", "explicit"],
                    help="how each CG step applies K_F (explicit: operator formed once per QP)")
    ap.add_argument("--poll", type=int, default=0,
                    help="CG steps between host polls (options.poll_every; 0: the library's adaptive chunks)")
    ap.add_argument("--cg-graph", type=int, default=0, choices=[0, 1],
                    help="1: replay each poll chunk of CG steps as a captured hipGraph (single-QP workloads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=0,
                    help="0: time one whole oracle solve; k > 0: k IPM iterations extrapolated")
    ap.add_argument("--no-batch-legs", action="store_true",
                    help="skip the 512-QP batched legs that the default workload reports beside its headline")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--single-count", type=int, default=512)
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--serve-warmup", type=int, default=10)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--shared-k", type=int, default=16, help="QPs of the shared workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (independent QPs shard "
              "across GPUs with no exchange; bench.py measures one GPU).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "mixed"
        return run_batch_workload(args)
    if args.workload == "serve":
        if args.precision == "fp64" and "--precision" not in sys.argv:
            args.precision = "mixed"
        return run_serve_workload(args)
    if args.workload == "shared":
        return run_shared_workload(args)

    import numpy as np
    import torch
    import synth
    from paper_2104_12916_amd import qpgpu

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload]
    prec_name = args.prec or w["prec"]
    prec = {"PL": qpgpu.QP_PREC_LOW_DOF, "PH": qpgpu.QP_PREC_FEW_EQ, "none": qpgpu.QP_PREC_NONE,
            "auto": qpgpu.QP_PREC_AUTO}[prec_name]
    precision = qpgpu.QP_MIXED if args.precision == "mixed" else qpgpu.QP_FP64
    kf = qpgpu.QP_KF_EXPLICIT if args.kf == "explicit" else qpgpu.QP_KF_IMPLICIT
    seeds = w["seeds"][:max(1, min(len(w["seeds"]), args.steps))]
    qps, solvers = [], []
    for sd in seeds:
        qp = synth.workload(args.workload, seed=sd)
        qps.append(qp)
        solvers.append(qpgpu.Solver(*qp.arrays(), prec=prec, precision=precision, profile=0 if args.cg_graph else 1,
                                    kf_form=kf, cg_graph=args.cg_graph, poll_every=args.poll))
    torch.cuda.synchronize()

    factor_s = []

    def step(i):
        s = solvers[i % len(solvers)]
        torch.cuda.synchronize()
        tf = time.perf_counter()
        s.factor()
        factor_s.append(time.perf_counter() - tf)
        x, lam, nu, sl, info = s.ipm(accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))
        return i % len(solvers), x, lam, nu, info

    for i in range(args.warmup):
        step(i)
        print(f"warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    for s in solvers:
        s.profile(reset=True)
    factor_s.clear()
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

    # parity of every timed solve: the KKT score and objective the library reports for the
    # returned iterate (pinned to the oracle's in tests/), the objective against the stored
    # oracle value
    ok = 0
    worst_kkt, worst_obj = 0.0, 0.0
    ipm_iters, cg_iters = [], []
    for k, x, lam, nu, info in outs:
        sc, f = info.rel_kkt, info.obj
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
    one_pass = solvers[0].k0_one_pass()
    names = OP_NAMES_ONE_PASS if one_pass else OP_NAMES
    tags = ["C^T", "M1" if one_pass else "M", "M1red" if one_pass else "M^T", "q", "XP", "XP^T"]
    if one_pass:  # M is read once; the partial sums are workspace, not operator bytes
        nbytes[2] = 0
        if qp0.m2 <= ONE_PASS_MAX:  # so is X_P in the P_H apply
            nbytes[5] = 0
        else:
            names = names[:4] + OP_NAMES[4:]
    if kf == qpgpu.QP_KF_EXPLICIT:  # one sweep over E (m2 x m2) replaces the four operator sweeps
        nbytes = [0, 0, 0, qp0.m2 * qp0.m2 * elem] + nbytes[4:]
    ops = {}
    for o in range(6):
        if cnt[o] > 0:
            ops[names[o]] = dict(avg_us=round(avg_ms[o] * 1e3, 2), samples=int(cnt[o]),
                                 bytes=nbytes[o], gbs=round(nbytes[o] / (avg_ms[o] * 1e-3) / 1e9, 1))
    dom = int(np.argmax(avg_ms))
    if avg_ms[dom] <= 0:  # no samples (graph replay takes none)
        avg_ms[dom] = float("nan")
    achieved = nbytes[dom] / (avg_ms[dom] * 1e-3) / 1e9
    traffic, tnote = load_traffic(args.workload, tags[dom])
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=names[dom],
                    bytes_per_launch=nbytes[dom], avg_launch_us=round(avg_ms[dom] * 1e3, 2),
                    traffic_note=tnote)
    # practical ceiling: the read rate of a plain streaming kernel over 2 GiB (8x the last-level cache)
    probe = {}
    for wg in (4, 8, 16):
        probe[wg] = (2 << 30) / (min(qpgpu.hbm_read_time(2 << 30, wg, 10) for _ in range(3)) * 1e-3) / 1e9
    best = max(probe, key=probe.get)
    roofline["measured_read_peak"] = dict(
        value=round(probe[best], 1), unit="GB/s", frac=round(achieved / probe[best], 4),
        probe=f"qp_hbm_read_time: 2 GiB, 16-byte non-temporal loads, {best} workgroups per CU (best of 4, 8, 16)")

    # CG steps of every reduced solve of one headline solve beside the theorem bound
    pred, corr = solvers[0].cg_steps()
    if prec == qpgpu.QP_PREC_LOW_DOF:
        bound, thm = min(qp0.m2, qp0.n - qp0.m1) + 1, "thm1 / cor:cg1 (P_L): min(m2, n - m1) + 1"
    elif prec == qpgpu.QP_PREC_FEW_EQ:
        bound, thm = min(qp0.m2, qp0.m1) + 1, "thm2 / cor:cg2 (P_H): min(m2, m1) + 1"
    else:
        bound, thm = qp0.m2, "no preconditioner: m2"
    cg_per_iter = dict(seed=seeds[0], predictor=pred, corrector=corr, bound=bound, theorem=thm,
                       over_bound=sum(int(k > bound) for k in pred + corr), solves=len(pred) + len(corr),
                       note="exact-arithmetic bound; the late IPM iterations' ill-conditioned systems need more "
                            "steps in float64")

    cpu = None
    if not args.no_cpu_baseline:
        if args.cpu_sample_iters > 0:
            cpu = cpu_baseline(args.workload, seeds[0], args.cpu_sample_iters, ipm_iters[0])
        else:
            cpu = cpu_baseline_full(args.workload, seeds[0])

    batch = None
    if args.workload == "lowdof" and not args.no_batch_legs:
        batch = config4_legs(args.batch_count, single=args.single_count > 0)

    # a0 (and a0' for P_H): algorithmic flops of the once-per-QP factorization over its wall time
    n, m1, m2 = qp0.n, qp0.m1, qp0.m2
    fl = n ** 3 / 3 + n * n * m1 + n * m1 * m1 + m1 ** 3 / 3
    if prec == qpgpu.QP_PREC_FEW_EQ:
        fl += n * n * m2 + m2 * m2 * n
    if kf == qpgpu.QP_KF_EXPLICIT:
        fl += (n * n / 2 + m1 * n) * m2 + m2 * m2 * (n + m1)  # Y = M C^T and E = Y1^T Y1 - Y2^T Y2
    fl *= 2  # multiply-adds
    f_ms = 1e3 * sum(factor_s) / max(1, len(factor_s))
    factor = dict(ms=round(f_ms, 3), algorithmic_gflop=round(fl / 1e9, 2),
                  tflops=round(fl / (f_ms * 1e-3) / 1e12, 2) if f_ms > 0 else None,
                  mfma_fp64_peak_tflops=78.6,
                  note="K0 = L Sigma L^T and its inverse factor (+ C H^-1 C^T for P_H); flops counted as the "
                       "factorization alone (the inverse triangles are extra work not counted)")
    value = ok / elapsed
    line = {
        "metric": METRIC, "value": value, "unit": "QP solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if precision == qpgpu.QP_MIXED else "f64",
        "data": "synthetic (seeded dense Gaussian QPs resident in HBM)",
        "config": {"workload": f"{args.workload}: {w['desc']}", "seeds": seeds, "precond": prec_name,
                   "precision": args.precision, "kf_form": args.kf, "cg_graph": args.cg_graph, "poll": args.poll},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": dict(passed=ok, solves=len(outs), max_rel_kkt=worst_kkt, max_obj_rel_err=worst_obj),
        "ipm_iters": ipm_iters, "cg_iters": cg_iters, "cg_per_ipm_iter": cg_per_iter,
        "us_per_cg_step": round(elapsed / max(1, sum(cg_iters)) * 1e6, 2),
        "us_per_ipm_iter": round(elapsed / max(1, sum(ipm_iters)) * 1e6, 1),
        "factor": factor,
        "cg_step_sweeps": ops,
        "batch": batch,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""CG steps per IPM iteration on the SyQP^n_{m1} family (the experiment of Sec. 6.2).

Generates SyQP^n_1 .. SyQP^n_n sharing one Hessian (block-diagonal 4 x 4 M^T M
blocks, banded A, C = I, d = 0; Sec. 6.1), solves each with the library's IPM in
float64 under four preconditioners -- none (U-KF), P_L (PL-KF), P_H with H
(PH-KF, eq. preconditioner-2) and P_H with diag(H) (the PH-KF form of Sec. 5.2)
-- and reports, per m1, the median CG steps of the reduced solves (predictor and
corrector of every IPM iteration) next to the exact-arithmetic bounds
min(m2, n - m1) + 1 (P_L, Theorem thm1) and min(m2, m1) + 1 (P_H, Theorem thm2).

Usage: python -m paper_2104_12916_amd.syqp_sweep [--n 64] [--step 1] [--json OUT]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

VARIANTS = [("U-KF", 0, 0), ("PL-KF", 1, 0), ("PH-KF", 2, 0), ("PH-KF diag(H)", 2, 1)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--step", type=int, default=1, help="sweep m1 = 1, 1 + step, ..., n")
    ap.add_argument("--json", default="")
    args = ap.parse_args()

    import numpy as np
    import synth
    from paper_2104_12916_amd import qpgpu

    n = args.n
    rows = []
    t0 = time.perf_counter()
    m1s = list(range(1, n + 1, args.step))
    if m1s[-1] != n:
        m1s.append(n)
    for m1 in m1s:
        qp = synth.syqp(m1, n, m1, H_seed=0)
        row = dict(m1=m1, bound_PL=min(qp.m2, n - m1) + 1, bound_PH=min(qp.m2, m1) + 1)
        for name, prec, form in VARIANTS:
            s = qpgpu.Solver(*qp.arrays(), prec=prec, ph_form=form)
            s.factor()
            x, lam, nu, sl, info = s.ipm(accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))
            k1, k2 = s.cg_steps()
            s.close()
            steps = k1 + k2
            row[name] = dict(median=float(np.median(steps)) if steps else 0.0, max=max(steps) if steps else 0,
                             ipm_iters=info.ipm_iters, rel_kkt=info.rel_kkt, status=info.status)
        rows.append(row)
        print(f"m1 {m1:3d}  " + "  ".join(f"{v[0]} {row[v[0]]['median']:6.1f}" for v in VARIANTS) +
              f"   bounds PL {row['bound_PL']} PH {row['bound_PH']}", flush=True)
    half = [r for r in rows if r["m1"] >= n / 2]
    summary = dict(
        n=n, seconds=round(time.perf_counter() - t0, 1),
        ph_below_unpreconditioned=sum(r["PH-KF"]["median"] < r["U-KF"]["median"] for r in rows) / len(rows),
        pl_below_unpreconditioned_m1_ge_half=sum(r["PL-KF"]["median"] < r["U-KF"]["median"] for r in half) /
        max(1, len(half)),
        ph_median_within_bound=sum(r["PH-KF"]["median"] <= r["bound_PH"] for r in rows) / len(rows),
        pl_median_within_bound_m1_gt_half=sum(r["PL-KF"]["median"] <= r["bound_PL"] for r in rows
                                               if r["m1"] > n / 2) / max(1, sum(r["m1"] > n / 2 for r in rows)),
        # the line the paper draws for P_L, 2 (n - m1) + 1
        pl_median_within_2nd_line_m1_gt_half=sum(r["PL-KF"]["median"] <= 2 * (n - r["m1"]) + 1 for r in rows
                                                 if r["m1"] > n / 2) / max(1, sum(r["m1"] > n / 2 for r in rows)),
        all_converged=all(r[v[0]]["status"] == 0 for r in rows for v in VARIANTS),
    )
    print(json.dumps(summary), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(dict(summary=summary, rows=rows), f, indent=1)


if __name__ == "__main__":
    main()

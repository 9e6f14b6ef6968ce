"""Autotuner of the streaming kernels' launch shapes (writes the library's cache).

For each size bucket n <= N (default N = 512, 1024, 2048, 4096) it builds a
seeded dense Gaussian QP of the low-dof shape (m1 = 3n/4, m2 = n/2), factorizes
it, and minimizes the device time of one whole P_L CG step (qp_op_time op 4: the
C^T p sweep, the one-pass K0 product, q = C w + D p and the update, or the
folded step when cg_fold is set) over the
kernel-shape keys by coordinate descent (two passes; every timing is the median
of three).  Larger n use the base entry.  The result goes to
autotune_gfx950.txt beside libqpgpu.so (or --out), which the library reads at
start-up (QPGPU_AUTOTUNE_CACHE overrides the path, QPGPU_TUNE the base entry).

Usage: python -m paper_2104_12916_amd.autotune [--buckets 512,1024,2048,4096] [--reps 30] [--out PATH]
"""
import argparse
import datetime
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

SPACE = [
    ("rows_bpc", [2, 4, 6, 8]),
    ("rows_unroll", [4, 8, 16]),
    ("sym_wg", [1, 2, 3, 4]),
    ("sym_units", [1, 4, 8, 16]),
    ("sym_teams", [1, 2]),
    ("sym_rows", [2, 4]),
    ("sym_pipe", [0, 1]),
    ("ld_nt", [0, 1, 2, 3]),
    ("upd_threads", [256, 512, 1024]),
    ("cg_fold", [2, 3]),  # bit 0 (P_L) is tuned; P_H stays folded
]


def spec(cfg):
    return ",".join(f"{k}={v}" for k, v in cfg.items())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--buckets", default="512,1024,2048,4096")
    ap.add_argument("--reps", type=int, default=30)
    ap.add_argument("--out", default="")
    args = ap.parse_args()

    import synth
    from paper_2104_12916_amd import qpgpu

    base_line = qpgpu.tune_get().splitlines()[0]  # "default ..." as loaded (built-in, env or cache)
    base = dict(kv.split("=") for kv in base_line.split(" ", 1)[1].split(","))
    start = {k: int(base[k]) for k, _ in SPACE}
    buckets = [int(b) for b in args.buckets.split(",")]
    chosen = {}
    for nmax in buckets:
        n = nmax
        qp = synth.gaussian_qp(7000 + n, n, 3 * n // 4, n // 2)
        s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_LOW_DOF)
        s.factor()

        def timed(cfg):
            qpgpu.tune_set(f"{base_line}\nn<={nmax} {spec(cfg)}")
            return statistics.median(s.op_time(4, qpgpu.QP_FP64, args.reps) for _ in range(3))

        cur = dict(start)
        best = timed(cur)
        first = best
        for _ in range(2):
            for key, values in SPACE:
                for v in values:
                    if v == cur[key]:
                        continue
                    cand = dict(cur, **{key: v})
                    t = timed(cand)
                    if t < best * 0.995:  # keep a change only for a clear gain
                        best, cur = t, cand
        s.close()
        chosen[nmax] = cur
        print(f"n<={nmax}: CG step {first * 1e3:.2f} -> {best * 1e3:.2f} us  {spec(cur)}", flush=True)
    qpgpu.tune_set(base_line)
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(qpgpu.LIB_PATH)), "autotune_gfx950.txt")
    lines = ["# Launch shapes per size bucket, chosen by paper_2104_12916_amd/autotune.py",
             f"# ({datetime.date.today()}; objective: one P_L CG step, qp_op_time op 4, low-dof shape"
             " m1 = 3n/4, m2 = n/2)",
             "arch gfx950", base_line]
    lines += [f"n<={nmax} {spec(cfg)}" for nmax, cfg in sorted(chosen.items())]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()

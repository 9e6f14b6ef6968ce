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

With --batch K it also tunes the base entry's keys of the batched kernels
(BATCH_SPACE) on a batch of the first K QPs of the 512-QP mix (n ~ U{64..1024},
m1 = n/4, m2 = n/2, seeds 1000+i; the preconditioner of the smaller CG bound),
minimizing the time of one whole batched solve (admission, factorizations and
every IPM iteration; median of three, one pass of coordinate descent).  Batches
use the base entry; single-QP calls use it only above the largest bucket.
--buckets "" keeps the loaded bucket entries.

Usage: python -m paper_2104_12916_amd.autotune [--buckets 512,1024,2048,4096] [--reps 30]
                                               [--batch K] [--batch-precision fp64|mixed] [--out PATH]
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


# keys of the batched kernels (row sweeps, one-pass sweep) in the base entry
BATCH_SPACE = [
    ("brows_unroll", [4, 8]),
    ("brows_stage", [0, 1]),
    ("bsym_units", [8, 16, 32]),
    ("bsym_wave", [0, 1]),
    ("sym_pipe", [0, 1]),
    ("sym_rows", [2, 4]),
    ("ld_nt", [0, 1, 2, 3]),
]


def spec(cfg):
    return ",".join(f"{k}={v}" for k, v in cfg.items())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--buckets", default="512,1024,2048,4096")
    ap.add_argument("--reps", type=int, default=30)
    ap.add_argument("--batch", type=int, default=0, help="tune the base entry on a batch of this many QPs")
    ap.add_argument("--batch-precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--out", default="")
    args = ap.parse_args()

    if args.batch > 0:
        # torch (device buffers of the batch) first: the library then shares its HIP runtime
        import torch
        torch.cuda.set_device(0)
    import synth
    from paper_2104_12916_amd import qpgpu

    loaded = qpgpu.tune_get().splitlines()
    base_line = loaded[0]  # "default ..." as loaded (built-in, env or cache)
    base = dict(kv.split("=") for kv in base_line.split(" ", 1)[1].split(","))
    start = {k: int(base[k]) for k, _ in SPACE}
    buckets = [int(b) for b in args.buckets.split(",") if b.strip()]
    chosen = {}
    if not buckets:  # keep the loaded bucket entries
        for ln in loaded[1:]:
            head, kv = ln.split(" ", 1)
            chosen[int(head[3:])] = dict(x.split("=") for x in kv.split(","))
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
    notes = []
    if args.batch > 0:
        bucket_lines = [f"n<={nmax} {spec(cfg)}" for nmax, cfg in sorted(chosen.items())]
        base_line, note = tune_batch(args, base_line, bucket_lines, qpgpu, synth)
        notes.append(note)
        qpgpu.tune_set(base_line)
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(qpgpu.LIB_PATH)), "autotune_gfx950.txt")
    lines = ["# Launch shapes per size bucket, chosen by paper_2104_12916_amd/autotune.py",
             f"# ({datetime.date.today()}; objective: one P_L CG step, qp_op_time op 4, low-dof shape"
             " m1 = 3n/4, m2 = n/2)"] + [f"# {x}" for x in notes] + ["arch gfx950", base_line]
    lines += [f"n<={nmax} {spec(cfg)}" for nmax, cfg in sorted(chosen.items())]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out}", flush=True)


def tune_batch(args, base_line, bucket_lines, qpgpu, synth):
    """Coordinate descent over BATCH_SPACE in the base entry; returns the new
    default line and a note on the gain."""
    import time
    import torch
    sizes = synth.batch_sizes(512, 1000)[:args.batch]
    dev = [tuple(torch.from_numpy(a).cuda() for a in synth.gaussian_qp(*sz).arrays()) for sz in sizes]
    precision = qpgpu.QP_FP64 if args.batch_precision == "fp64" else qpgpu.QP_MIXED
    opt = qpgpu.qp_default_options(prec=qpgpu.QP_PREC_AUTO, precision=precision)
    budget = int(1.05 * sum(qpgpu.qp_batch_footprint(opt, *sz[1:]) for sz in sizes)) + (64 << 20)
    base = dict(kv.split("=") for kv in base_line.split(" ", 1)[1].split(","))

    def solve():
        b = qpgpu.Batch(budget, prec=qpgpu.QP_PREC_AUTO, precision=precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = [b.admit(*d) for d in dev]
        if any(tk is None for tk in tickets):
            raise RuntimeError("batch budget too small")
        while b.query()["in_flight"]:
            b.step(1)
        for tk in tickets:
            b.collect(tk, accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        b.close()
        return el

    def line(cfg):
        return "default " + ",".join(f"{k}={cfg.get(k, v)}" for k, v in base.items())

    def timed(cfg):
        qpgpu.tune_set("\n".join([line(cfg)] + bucket_lines))
        return statistics.median(solve() for _ in range(3))

    cur = {k: int(base[k]) for k, _ in BATCH_SPACE}
    solve()  # warm-up
    best = first = timed(cur)
    for key, values in BATCH_SPACE:
        for v in values:
            if v == cur[key]:
                continue
            cand = dict(cur, **{key: v})
            t = timed(cand)
            print(f"batch {spec(cand)}: {t * 1e3:.1f} ms", flush=True)
            if t < best * 0.98:  # keep a change only for a clear gain
                best, cur = t, cand
    note = (f"base entry's batched keys on {len(dev)} QPs of the batched mix ({args.batch_precision}): "
            f"{first * 1e3:.0f} -> {best * 1e3:.0f} ms per batch, {spec(cur)}")
    print(note, flush=True)
    return line(cur), note


if __name__ == "__main__":
    main()

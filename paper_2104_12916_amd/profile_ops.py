"""Kernel-level timing run for profilers (rocprofv3 --kernel-trace / --pmc).

Sets up one workload instance, factorizes it, then launches each CG-step sweep
`reps` times through qp_op_time (same kernels and launch shapes as inside the
solver) and, for counter calibration, one plain device-to-device copy of a known
size.  Prints the event-timed averages.

With --dense N it times the factorization kernels instead (qp_dense_time): the
n^3 GEMM, the GEMM with a triangular operand and the Cholesky-inverse of size N,
with their rates (flops of the product, of the Cholesky alone for op 2).

With --shared K it runs the block PCG of K QPs sharing the low-dof instance's H, A
and C (qp_shared_pcg_solve, P_L, a fixed number of steps: --reps) twice, for a
kernel trace of the multi-vector MFMA sweeps; it prints each sweep's matrix bytes.

Usage: python -m paper_2104_12916_amd.profile_ops [--workload lowdof] [--reps 10] [--dense N] [--shared K]
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_BYTES = 256 << 20


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="lowdof")
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--dense", type=int, default=0, help="time the factorization kernels of this size")
    ap.add_argument("--shared", type=int, default=0, help="block PCG over this many QPs sharing H, A, C")
    args = ap.parse_args()

    if args.shared:
        import time
        import numpy as np
        import synth
        from paper_2104_12916_amd import qpgpu
        qp = synth.workload("lowdof", seed=100)
        n, m1, m2, k = qp.n, qp.m1, qp.m2, args.shared
        sh = qpgpu.Shared(qp.H, qp.A, qp.C, prec=qpgpu.QP_PREC_LOW_DOF)
        rng = np.random.default_rng(0)
        dv, rh = rng.uniform(0.5, 2.0, (k, m2)), rng.standard_normal((k, m2))
        mm = (n * (n + 1) // 2 + m1 * n) * 8
        print(f"shared block PCG: k={k}, {args.reps} steps per run; matrix bytes per sweep: C^T {n * m2 * 8}, "
              f"M {mm}, M^T {mm}, C {m2 * n * 8}", flush=True)
        for r in range(2):
            t0 = time.perf_counter()
            sh.pcg(dv, rh, rtol=1e-300, maxit=args.reps, accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))
            dt = time.perf_counter() - t0
            print(f"run {r}: {dt * 1e3:.1f} ms, {dt / args.reps * 1e6:.1f} us per block step", flush=True)
        sh.close()
        return

    if args.dense:
        from paper_2104_12916_amd import qpgpu
        n = args.dense
        for op, name, flops in ((0, "GEMM C = A B^T", 2.0 * n ** 3), (1, "GEMM, B^T upper triangular", 1.0 * n ** 3),
                                (2, "Cholesky-inverse", 2.0 * n ** 3 / 3.0)):
            ms = qpgpu.dense_time(op, n, args.reps)
            print(f"dense op {op} ({name}), n={n}: {ms:.3f} ms, {flops / (ms * 1e-3) / 1e12:.1f} TF/s "
                  f"({100 * flops / (ms * 1e-3) / 78.6e12:.1f} % of 78.6)", flush=True)
        return

    import torch
    import synth
    from paper_2104_12916_amd import qpgpu

    torch.cuda.set_device(0)
    qp = synth.workload(args.workload, seed=args.seed)
    mixed = args.precision == "mixed"
    s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_LOW_DOF,
                     precision=qpgpu.QP_MIXED if mixed else qpgpu.QP_FP64)
    s.factor()
    # calibration copy: COPY_BYTES read and COPY_BYTES written by one elementwise kernel
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy kernel: {COPY_BYTES} bytes read, {COPY_BYTES} bytes written", flush=True)
    names = ["C^T p", "Sigma M u", "M^T v", "C w", "CG step"]
    if s.k0_one_pass():
        names[1:3] = ["one-pass M^T Sigma M u sweep", "sum of its partials"]
    for op in range(5):
        ms = s.op_time(op, qpgpu.QP_MIXED if mixed else qpgpu.QP_FP64, args.reps)
        print(f"op {op} ({names[op]}): {ms * 1e3:.2f} us per launch", flush=True)
    s.close()


if __name__ == "__main__":
    main()

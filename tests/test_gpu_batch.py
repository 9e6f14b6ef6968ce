"""Batches of independent QPs through qp_batch_* (needs an MI355X).

Every batched result is checked against the oracle (its relative KKT score of
the GPU iterate <= 1e-8 and the objective within 1e-7 * max(1, |f*|) of the
oracle's full-KKT IPM), and a QP's result must not depend on the other QPs of
its batch: each QP's launch shapes and arithmetic depend only on that QP, so
the iterate is compared bit for bit between a batch of one and a mixed batch.
"""
import numpy as np
import pytest

import synth
from oracle import ipm, kkt
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu

PL, PH, AUTO = qpgpu.QP_PREC_LOW_DOF, qpgpu.QP_PREC_FEW_EQ, qpgpu.QP_PREC_AUTO


def mixed_sizes(count, seed, n_lo=16, n_hi=300):
    """(seed_i, n, m1, m2) with n ~ U{n_lo..n_hi}, m1 = n // 4, m2 = n // 2 (ragged tiles)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        out.append((seed + i, n, max(1, n // 4), max(1, n // 2)))
    return out


def instances(sizes):
    return [synth.gaussian_qp(s, n, m1, m2) for (s, n, m1, m2) in sizes]


def run_batch(qps, budget=0, rounds=1000, **opts):
    b = qpgpu.Batch(budget, **opts)
    tickets = [b.admit(*qp.arrays()) for qp in qps]
    assert all(t is not None for t in tickets)
    b.step(rounds)
    done = set(b.finished())
    assert done == set(tickets)
    out = [b.collect(t) for t in tickets]
    q = b.query()
    assert q["in_flight"] == 0 and q["finished"] == 0 and q["bytes_used"] == 0
    b.close()
    return out


def _check_reported(qp, x, lam, nu, info):
    """The KKT score and objective the library reports for its returned iterate
    (computed in float64 on the GPU) agree with the oracle's on the same iterate."""
    sc, _ = kkt.rel_kkt(qp, x, lam, nu)
    assert abs(info.rel_kkt - sc) <= 1e-12 + 1e-6 * sc, (info.rel_kkt, sc)
    f = kkt.objective(qp, x)
    assert abs(info.obj - f) <= 1e-10 * max(1.0, abs(f)), (info.obj, f)


def check_against_oracle(qp, x, lam, nu, f_ref):
    score, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert score <= 1e-8, parts
    f = kkt.objective(qp, x)
    assert abs(f - f_ref) <= 1e-7 * max(1.0, abs(f_ref))


@pytest.mark.parametrize("prec,precision", [(PH, qpgpu.QP_FP64), (PL, qpgpu.QP_FP64), (AUTO, qpgpu.QP_MIXED),
                                            (PH, qpgpu.QP_MIXED)])
def test_batch_matches_oracle(gpu, prec, precision):
    qps = instances(mixed_sizes(10, 1000 + 17 * prec + precision))
    res = run_batch(qps, prec=prec, precision=precision)
    for qp, (x, lam, nu, s, info) in zip(qps, res):
        ref = ipm.solve(qp)
        assert ref.converged
        check_against_oracle(qp, x, lam, nu, ref.obj)
        _check_reported(qp, x, lam, nu, info)
        assert np.all(nu > 0) and np.all(s > 0)
        assert info.status == qpgpu.QP_OK and info.ipm_iters <= ref.iters + 10
        assert info.t_solve_ms > 0


def test_batch_result_alone_equals_result_in_mix(gpu):
    qps = instances(mixed_sizes(7, 3100))
    mix = run_batch(qps, prec=AUTO, precision=qpgpu.QP_MIXED)
    for qp, (x, lam, nu, s, info) in zip(qps, mix):
        (xa, la, na, sa, ia), = run_batch([qp], prec=AUTO, precision=qpgpu.QP_MIXED)
        assert np.array_equal(x, xa) and np.array_equal(lam, la) and np.array_equal(nu, na)
        assert np.array_equal(s, sa)
        assert info.ipm_iters == ia.ipm_iters and info.pcg_iters_total == ia.pcg_iters_total


def test_batch_agrees_with_single_qp_path(gpu):
    qps = instances(mixed_sizes(4, 3200))
    res = run_batch(qps, prec=PH)
    for qp, (x, lam, nu, s, info) in zip(qps, res):
        solo = qpgpu.Solver(*qp.arrays(), prec=PH)
        solo.factor()
        xs, ls, ns, ss, si = solo.ipm()
        solo.close()
        # same method, different launch shapes (rounding order): agreement to the IPM tolerance
        f, fs = kkt.objective(qp, x), kkt.objective(qp, xs)
        assert abs(f - fs) <= 1e-7 * max(1.0, abs(fs))
        assert abs(info.ipm_iters - si.ipm_iters) <= 2


def test_batch_admission_by_memory(gpu):
    qps = instances(mixed_sizes(9, 3300, 40, 200))
    opt = qpgpu.qp_default_options(prec=PH)
    sizes = [qpgpu.qp_batch_footprint(opt, qp.n, qp.m1, qp.m2) for qp in qps]
    assert all(s > 0 for s in sizes)
    budget = sum(sorted(sizes)[-3:])  # room for about three QPs at a time
    b = qpgpu.Batch(budget, prec=PH)
    pending = list(range(len(qps)))
    tickets = {}
    refused = 0
    rounds = 0
    while pending or b.query()["in_flight"]:
        while pending:
            t = b.admit(*qps[pending[0]].arrays())
            if t is None:
                refused += 1
                break
            tickets[t] = pending.pop(0)
        assert b.query()["bytes_used"] <= budget
        b.step(1)
        rounds += 1
        assert rounds < 2000
    assert refused > 0  # the budget did bind
    for t in b.finished():
        qp = qps[tickets[t]]
        x, lam, nu, s, info = b.collect(t)
        check_against_oracle(qp, x, lam, nu, ipm.solve(qp).obj)
    assert b.query()["bytes_used"] == 0
    b.close()


def test_batch_continuous_admission(gpu):
    qps = instances(mixed_sizes(6, 3400))
    b = qpgpu.Batch(0, prec=AUTO, precision=qpgpu.QP_MIXED)
    t1 = [b.admit(*qp.arrays()) for qp in qps[:3]]
    b.step(3)
    assert b.query()["in_flight"] > 0
    t2 = [b.admit(*qp.arrays()) for qp in qps[3:]]
    b.step(1000)
    assert set(b.finished()) == set(t1 + t2)
    for qp, t in zip(qps, t1 + t2):
        x, lam, nu, s, info = b.collect(t)
        check_against_oracle(qp, x, lam, nu, ipm.solve(qp).obj)
    b.close()


def test_batch_failures_are_isolated(gpu):
    good = instances(mixed_sizes(3, 3500, 30, 80))
    bad_rank = synth.gaussian_qp(7, 30, 6, 12)
    A = bad_rank.A.copy()
    A[1] = A[0]  # rank-deficient equality block
    bad_spd = synth.gaussian_qp(8, 25, 5, 10)
    Hn = bad_spd.H - 2.0 * np.linalg.norm(bad_spd.H, 2) * np.eye(25)  # symmetric, not positive definite
    b = qpgpu.Batch(0, prec=AUTO)
    tg = [b.admit(*qp.arrays()) for qp in good]
    tr = b.admit(bad_rank.H, bad_rank.c, np.ascontiguousarray(A), bad_rank.b, bad_rank.C, bad_rank.d)
    ts = b.admit(np.ascontiguousarray(Hn), bad_spd.c, bad_spd.A, bad_spd.b, bad_spd.C, bad_spd.d)
    b.step(1000)
    _, _, _, _, ir = b.collect(tr, accept=(qpgpu.QP_E_RANK,))
    assert ir.status == qpgpu.QP_E_RANK
    _, _, _, _, isp = b.collect(ts, accept=(qpgpu.QP_E_NOT_SPD,))
    assert isp.status == qpgpu.QP_E_NOT_SPD
    for qp, t in zip(good, tg):
        x, lam, nu, s, info = b.collect(t)
        check_against_oracle(qp, x, lam, nu, ipm.solve(qp).obj)
    b.close()


def test_batch_call_order_and_tickets(gpu):
    qp = synth.gaussian_qp(11, 40, 10, 20)
    b = qpgpu.Batch(0)
    t = b.admit(*qp.arrays())
    x, lam, nu, s = np.zeros(40), np.zeros(10), np.zeros(20), np.zeros(20)
    st, _ = qpgpu.qp_batch_collect(b.b, t, x, lam, nu, s)
    assert st == qpgpu.QP_E_STATE  # not finished yet
    st, _ = qpgpu.qp_batch_collect(b.b, t + 1000, x, lam, nu, s)
    assert st == qpgpu.QP_E_INVALID
    b.step(1000)
    st, _ = qpgpu.qp_batch_collect(b.b, t, x, lam, nu, s)
    assert st == qpgpu.QP_OK
    st, _ = qpgpu.qp_batch_collect(b.b, t, x, lam, nu, s)
    assert st == qpgpu.QP_E_INVALID  # collected tickets are forgotten
    # stepping an empty batch is a no-op
    assert b.step(5) == 0
    b.close()


def test_batch_degenerate_and_equal_sizes(gpu):
    # one-variable QPs, m1 = n (K_F = D) and identical sizes side by side
    qps = [synth.gaussian_qp(1, 1, 1, 1), synth.gaussian_qp(2, 6, 6, 4), synth.gaussian_qp(3, 33, 8, 16),
           synth.gaussian_qp(4, 33, 8, 16)]
    res = run_batch(qps, prec=AUTO)
    for qp, (x, lam, nu, s, info) in zip(qps, res):
        check_against_oracle(qp, x, lam, nu, ipm.solve(qp).obj)

"""The folded CG step against the step with a separate update kernel (needs an MI355X).

The folded step merges the vector update into the operator sweeps: p^T q comes
from u^T w + p^T D p (u = C^T p, w the K0 product), and for P_H the sum of the
X_P apply's partials also forms r^T z.  It is the same preconditioned CG with
those inner products summed differently, so both must reach the oracle's
solution of K_F dnu = r at the solve tolerance, with step counts that differ by
rounding only.  Bit 0 of the cg_fold key folds P_L solves, bit 1 P_H solves; bit 2 takes
C^T p_old in the folded C^T sweep from the previous step's u = C^T p, a recurrence
whose rounding must not cost accuracy or steps either.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import ipm as oracle_ipm
from oracle import kkt, reduced
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture
def table():
    before = qpgpu.tune_get()
    yield before
    qpgpu.tune_set(before)


# shapes where each preconditioner converges well (P_L needs many equalities, P_H few)
CASES = [(qpgpu.QP_PREC_LOW_DOF, 300, 200, 150), (qpgpu.QP_PREC_LOW_DOF, 700, 500, 333),
         (qpgpu.QP_PREC_FEW_EQ, 200, 50, 100), (qpgpu.QP_PREC_FEW_EQ, 900, 100, 900)]


@pytest.mark.parametrize("prec,n,m1,m2", CASES)
def test_folded_pcg_matches_separate_update(gpu, table, prec, n, m1, m2):
    base = table.splitlines()[0]
    qp = synth.gaussian_qp(6100 + n + prec, n, m1, m2)
    dvec = synth.log_uniform(31 + n, m2, 1e-2, 1e2)
    rhs = np.random.default_rng(n).standard_normal(m2)
    ref = sla.cho_solve(sla.cho_factor(reduced.kf_explicit(qp, dvec)), rhs)
    out = {}
    for fold in (0, 3, 7):
        qpgpu.tune_set(f"{base}\ndefault cg_fold={fold}")
        s = qpgpu.Solver(*qp.arrays(), prec=prec)
        s.factor()
        dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=1e-12)
        s.close()
        assert relerr(dnu, ref) <= 1e-8, fold
        assert info.rel_res <= 1e-11, fold
        out[fold] = info.iters
    for fold in (3, 7):
        assert abs(out[fold] - out[0]) <= max(2, out[0] // 10), out


@pytest.mark.parametrize("fold", [2, 6])
@pytest.mark.parametrize("precision", [qpgpu.QP_FP64, qpgpu.QP_MIXED])
def test_folded_ph_ipm_matches_oracle(gpu, table, precision, fold):
    """A whole P_H IPM with the folded step in both precisions, with C^T p_old from
    a second dot per row (cg_fold=2) and from the previous step's u (6)."""
    base = table.splitlines()[0]
    qpgpu.tune_set(f"{base}\ndefault cg_fold={fold}")
    qp = synth.gaussian_qp(6301, 400, 60, 400)
    s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_FEW_EQ, precision=precision)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    s.close()
    ref = oracle_ipm.solve(qp, tol=1e-10)
    assert ref.converged and info.status == qpgpu.QP_OK
    score, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert score <= 1e-8, parts
    assert abs(kkt.objective(qp, x) - ref.obj) <= 1e-7 * max(1.0, abs(ref.obj))

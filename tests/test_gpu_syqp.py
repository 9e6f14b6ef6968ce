"""The preconditioners on the paper's own family SyQP^64_{m1} (needs an MI355X).

SyQP^n_{m1} (Sec. 6.1): block-diagonal 4 x 4 M^T M Hessian shared over m1, banded
A, C = I, d = 0.  The GPU IPM (float64, C = I path) is checked against the oracle
for every preconditioner, and the CG steps it takes per reduced solve are checked
against what Sec. 6.2 reports for this family: P_H lowers the median below the
unpreconditioned CG for every m1 and keeps it within its bound m1 + 1 (Theorem
thm2); P_L lowers it for m1 >= n/2 and keeps it within the line 2 (n - m1) + 1 the
paper draws once m1 is not close to n/2.  (Exact termination at the bounds is not pinned on this family: its
nearly singular 4 x 4 blocks make P_H = D + H^{-1} so ill-conditioned that even
the oracle's PCG does not collapse there; the counts are medians over IPM
iterations, as in the paper.)
"""
import numpy as np
import pytest

import synth
from oracle import ipm, kkt
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu

N = 64
OK = (qpgpu.QP_OK,)


def solve(qp, prec, form=qpgpu.QP_PH_EXACT):
    s = qpgpu.Solver(*qp.arrays(), prec=prec, ph_form=form)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    k1, k2 = s.cg_steps()
    s.close()
    return x, lam, nu, info, k1, k2


@pytest.mark.parametrize("m1", [1, 17, 40, 63])
@pytest.mark.parametrize("prec,form", [(qpgpu.QP_PREC_NONE, 0), (qpgpu.QP_PREC_LOW_DOF, 0),
                                       (qpgpu.QP_PREC_FEW_EQ, 0), (qpgpu.QP_PREC_FEW_EQ, 1)])
def test_syqp_ipm_matches_oracle(gpu, m1, prec, form):
    qp = synth.syqp(m1, N, m1, H_seed=0)
    x, lam, nu, info, k1, k2 = solve(qp, prec, form)
    sc, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert sc <= 1e-8, parts
    f_ref = ipm.solve(qp).obj
    assert abs(kkt.objective(qp, x) - f_ref) <= 1e-7 * max(1.0, abs(f_ref))
    # the per-iteration trace adds up to the totals
    assert len(k1) == len(k2) == info.ipm_iters
    assert sum(k1) + sum(k2) == info.pcg_iters_total


@pytest.mark.parametrize("m1", [1, 5, 12, 24, 33, 40, 48, 56, 60, 64])
def test_syqp_cg_steps_per_preconditioner(gpu, m1):
    qp = synth.syqp(m1, N, m1, H_seed=0)
    med = {}
    for name, prec in (("U", qpgpu.QP_PREC_NONE), ("L", qpgpu.QP_PREC_LOW_DOF), ("H", qpgpu.QP_PREC_FEW_EQ)):
        *_, k1, k2 = solve(qp, prec)
        med[name] = float(np.median(k1 + k2))
    assert med["H"] < med["U"], med
    assert med["H"] <= min(N, m1) + 1, med
    if m1 >= N / 2:
        assert med["L"] < med["U"], med
    if m1 >= 40:  # just above n/2 (m1 = 33..38) rounding pushes P_L past the line, as Sec. 6.2 notes
        assert med["L"] <= 2 * (N - m1) + 1, med

"""Parity of the explicit reduced operator (QP_KF_EXPLICIT) against the oracle (needs an MI355X).

With QP_KF_EXPLICIT the library forms E = C K0^{-1}_{11} C^T once per QP and every
CG step applies K_F = D + E with one row sweep.  Same bars as the implicit path:
  * K_F product: normwise relative error <= max(1e-10, 100 eps cond(K0)) against
    the oracle's K_F (E is the same linear map; its rounding grows with cond(K0)
    like the implicit product's);
  * PCG at rtol 1e-12: <= 1e-8 against the Cholesky solution of the explicit K_F;
  * IPM: the oracle's relative KKT score of the GPU iterate <= 1e-8 and the
    objective within 1e-7 * max(1, |f*|) of the oracle's (golden values at full size).
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import ipm, kkt, reduced
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu

PL, PH, PN, AUTO = qpgpu.QP_PREC_LOW_DOF, qpgpu.QP_PREC_FEW_EQ, qpgpu.QP_PREC_NONE, qpgpu.QP_PREC_AUTO
EX = qpgpu.QP_KF_EXPLICIT
HERE = os.path.dirname(os.path.abspath(__file__))
SIZES = [(1, 1, 1), (5, 2, 3), (70, 30, 40), (200, 50, 100), (129, 65, 257), (300, 130, 170), (260, 259, 300)]


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def k0_tol(qp):
    return max(1e-10, 100 * np.finfo(float).eps * np.linalg.cond(reduced.K0_matrix(qp)))


def check_ipm(qp, x, lam, nu, f_ref):
    sc, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert sc <= 1e-8, parts
    f = kkt.objective(qp, x)
    assert abs(f - f_ref) <= 1e-7 * max(1.0, abs(f_ref))


@pytest.mark.parametrize("n,m1,m2", SIZES)
def test_explicit_kf_apply_matches_definition(gpu, n, m1, m2):
    qp = synth.gaussian_qp(2000 + n + m2, n, m1, m2)
    s = qpgpu.Solver(*qp.arrays(), kf_form=EX)
    s.factor()
    dvec = synth.log_uniform(5, m2, 1e-3, 1e3)
    p = np.random.default_rng(m2).standard_normal(m2)
    q = s.kf_apply(dvec, p)
    ref = reduced.kf_explicit(qp, dvec) @ p
    assert relerr(q, ref) <= k0_tol(qp)
    assert np.max(np.abs(q - ref)) <= k0_tol(qp) * np.max(np.abs(ref))  # element by element
    s.close()


@pytest.mark.parametrize("prec", [PL, PH, PN])
@pytest.mark.parametrize("n,m1,m2", [(5, 2, 3), (70, 30, 40), (200, 50, 100), (129, 65, 257), (300, 130, 170)])
def test_explicit_pcg_matches_direct_reduced_solve(gpu, prec, n, m1, m2):
    qp = synth.gaussian_qp(3000 + n, n, m1, m2)
    s = qpgpu.Solver(*qp.arrays(), kf_form=EX)
    s.factor()
    dvec = synth.log_uniform(9, m2, 1e-2, 1e2)
    rhs = np.random.default_rng(3).standard_normal(m2)
    dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=1e-12)
    ref = sla.cho_solve(sla.cho_factor(reduced.kf_explicit(qp, dvec)), rhs)
    assert relerr(dnu, ref) <= 1e-8
    assert info.rel_res <= 1e-11
    s.close()


@pytest.mark.parametrize("prec", [PL, PH])
@pytest.mark.parametrize("seed", list(range(8)))
def test_explicit_ipm_small_workload_matches_oracle(gpu, seed, prec):
    qp = synth.gaussian_qp(seed, 200, 50, 100)
    ref = ipm.solve(qp)
    s = qpgpu.Solver(*qp.arrays(), prec=prec, kf_form=EX)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    check_ipm(qp, x, lam, nu, ref.obj)
    assert info.ipm_iters <= ref.iters + 5
    s.close()


@pytest.mark.parametrize("prec", [PL, PH])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_explicit_mixed_ipm_matches_oracle(gpu, seed, prec):
    qp = synth.gaussian_qp(seed, 200, 50, 100)
    ref = ipm.solve(qp)
    s = qpgpu.Solver(*qp.arrays(), prec=prec, kf_form=EX, precision=qpgpu.QP_MIXED)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    check_ipm(qp, x, lam, nu, ref.obj)
    s.close()


def _batch(qps, **opts):
    b = qpgpu.Batch(0, **opts)
    tickets = [b.admit(*qp.arrays()) for qp in qps]
    b.step(100000)
    out = [b.collect(t) for t in tickets]
    b.close()
    return out


@pytest.mark.parametrize("precision", [qpgpu.QP_FP64, qpgpu.QP_MIXED])
def test_explicit_batch_matches_oracle_and_is_mix_independent(gpu, precision):
    rng = np.random.default_rng(77)
    qps = []
    for i in range(8):
        n = int(rng.integers(16, 260))
        qps.append(synth.gaussian_qp(7700 + i, n, max(1, n // 4), max(1, n // 2)))
    mix = _batch(qps, prec=AUTO, precision=precision, kf_form=EX)
    for qp, (x, lam, nu, s, info) in zip(qps, mix):
        check_ipm(qp, x, lam, nu, ipm.solve(qp).obj)
    (xa, la, na, sa, ia), = _batch([qps[3]], prec=AUTO, precision=precision, kf_form=EX)
    assert np.array_equal(xa, mix[3][0]) and np.array_equal(na, mix[3][2])


def _golden(workload, seed):
    with open(os.path.join(HERE, "golden", f"oracle_{workload}_{seed}.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("workload,seed,prec", [("lowdof", 100, PL), ("fewEq", 200, PH)])
def test_explicit_fullsize_ipm_matches_oracle(gpu, workload, seed, prec):
    qp = synth.workload(workload, seed=seed)
    g = _golden(workload, seed)
    s = qpgpu.Solver(*qp.arrays(), prec=prec, kf_form=EX)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    s.close()
    score, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert score <= 1e-8, parts
    f = kkt.objective(qp, x)
    assert abs(f - g["obj"]) <= 1e-7 * max(1.0, abs(g["obj"]))

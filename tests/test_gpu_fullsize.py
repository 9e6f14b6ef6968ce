"""Parity at the full sizes of the benchmarked workloads (needs an MI355X).

Same C-ABI calls and launch shapes as bench.py.  Where the oracle cannot
afford the whole computation it checks properties that hold at any size
(backward error of the K0 solve, the oracle's KKT score of the solution) or
one full product it can form with a single dense solve.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import kkt, reduced
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def golden(workload, seed):
    with open(os.path.join(HERE, "golden", f"oracle_{workload}_{seed}.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def lowdof():
    qp = synth.workload("lowdof", seed=100)
    s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_LOW_DOF)
    s.factor()
    yield qp, s
    s.close()


def test_fullsize_k0_solve_backward_error(gpu, lowdof):
    qp, s = lowdof
    rhs = np.random.default_rng(7).standard_normal(qp.n + qp.m1)
    out = s.k0_solve(rhs)
    x, y = out[:qp.n], out[qp.n:]
    resid = np.concatenate([qp.H @ x + qp.A.T @ y, qp.A @ x]) - rhs
    scale = (np.linalg.norm(qp.H, 2) + np.linalg.norm(qp.A, 2)) * np.linalg.norm(out) + np.linalg.norm(rhs)
    # backward error of a solve through an inverted factor: O(cond(L) eps); 1e-11 allows cond(L) ~ 1e4
    assert np.linalg.norm(resid) / scale <= 1e-11


def test_fullsize_kf_apply_matches_dense_solve(gpu, lowdof):
    qp, s = lowdof
    dvec = synth.log_uniform(3, qp.m2, 1e-3, 1e3)
    p = np.random.default_rng(8).standard_normal(qp.m2)
    q = s.kf_apply(dvec, p)
    ref = reduced.kf_apply(qp, dvec, p)
    assert np.linalg.norm(q - ref) / np.linalg.norm(ref) <= 1e-9
    # element by element, against the largest entry of the product
    assert np.max(np.abs(q - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_fullsize_pcg_true_residual(gpu, lowdof):
    qp, s = lowdof
    dvec = synth.log_uniform(4, qp.m2, 1e-2, 1e2)
    rhs = np.random.default_rng(9).standard_normal(qp.m2)
    dnu, info = s.pcg(dvec, rhs, prec=qpgpu.QP_PREC_LOW_DOF, rtol=1e-10)
    # residual with the oracle's K_F product (one dense K0 solve on the host)
    res = rhs - reduced.kf_apply(qp, dvec, dnu)
    assert np.linalg.norm(res) / np.linalg.norm(rhs) <= 1e-8
    assert info.iters <= 10 * qp.m2


def _check_reported(qp, x, lam, nu, info):
    """The KKT score and objective the library reports for its returned iterate
    (computed in float64 on the GPU) agree with the oracle's on the same iterate."""
    sc, _ = kkt.rel_kkt(qp, x, lam, nu)
    assert abs(info.rel_kkt - sc) <= 1e-12 + 1e-6 * sc, (info.rel_kkt, sc)
    f = kkt.objective(qp, x)
    assert abs(info.obj - f) <= 1e-10 * max(1.0, abs(f)), (info.obj, f)


def test_fullsize_lowdof_ipm_matches_oracle(gpu, lowdof):
    qp, s = lowdof
    g = golden("lowdof", 100)
    x, lam, nu, sl, info = s.ipm()
    score, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert score <= 1e-8, parts
    f = kkt.objective(qp, x)
    assert abs(f - g["obj"]) <= 1e-7 * max(1.0, abs(g["obj"]))
    assert info.ipm_iters <= g["iters"] + 10
    _check_reported(qp, x, lam, nu, info)  # the score bench.py counts solves by


@pytest.mark.parametrize("seed", [200, 201, 202])
def test_fullsize_fewEq_ipm_matches_oracle(gpu, seed):
    qp = synth.workload("fewEq", seed=seed)
    g = golden("fewEq", seed)
    s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_FEW_EQ)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    s.close()
    score, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert score <= 1e-8, parts
    f = kkt.objective(qp, x)
    assert abs(f - g["obj"]) <= 1e-7 * max(1.0, abs(g["obj"]))


def test_fullsize_lowdof_mixed_ipm_matches_oracle(gpu):
    qp = synth.workload("lowdof", seed=100)
    g = golden("lowdof", 100)
    s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_LOW_DOF, precision=qpgpu.QP_MIXED)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    s.close()
    score, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert score <= 1e-8, parts
    f = kkt.objective(qp, x)
    assert abs(f - g["obj"]) <= 1e-7 * max(1.0, abs(g["obj"]))

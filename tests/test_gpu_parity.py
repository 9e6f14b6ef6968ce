"""Parity of the HIP path against the CPU oracle (needs an MI355X).

Every call goes through the C ABI (ctypes binding).  Inputs are seeded
synthetic instances; expected values come from oracle/ only.

Tolerances (float64 throughout):
  * K0 solve and K_F product: normwise relative error <= max(1e-10,
    100 eps cond(K0)), and every entry within that bound times the largest
    entry of the reference.  Both sides compute the same linear map; the GPU
    applies inverted triangular factors, whose forward error, like that of a
    backward-stable solve, grows with cond(K0) * eps.
  * PCG at rtol 1e-12: relative error <= 1e-8 against the Cholesky solution of
    the explicit K_F (cond(K_F) <= ~1e4 for D in [1e-2, 1e2]).
  * IPM: the oracle's relative KKT score of the GPU output <= 1e-8 and the
    objective within 1e-7 * max(1, |f*|) of the oracle's.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import boxqp, bruteforce, ipm, kkt, reduced
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu

PL, PH, PN = qpgpu.QP_PREC_LOW_DOF, qpgpu.QP_PREC_FEW_EQ, qpgpu.QP_PREC_NONE

# sizes span several 64/128-wide tiles and ragged tails; (1, 1, 1) is the degenerate case
SIZES = [(1, 1, 1), (5, 2, 3), (70, 30, 40), (200, 50, 100), (129, 65, 257), (300, 130, 170), (260, 259, 300)]


def make(qp, **opts):
    return qpgpu.Solver(*qp.arrays(), **opts)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elemerr(a, b):
    """max_i |a_i - b_i| / max_i |b_i| (element-by-element bar)."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def k0_tol(qp):
    return max(1e-10, 100 * np.finfo(float).eps * np.linalg.cond(reduced.K0_matrix(qp)))


@pytest.mark.parametrize("n,m1,m2", SIZES)
def test_k0_solve_matches_dense_solve(gpu, n, m1, m2):
    qp = synth.gaussian_qp(1000 + n + m1, n, m1, m2)
    s = make(qp)
    s.factor()
    rhs = np.random.default_rng(n).standard_normal(n + m1)
    out = s.k0_solve(rhs)
    ref = reduced.k0_solve(qp, rhs)
    assert relerr(out, ref) <= k0_tol(qp)
    assert elemerr(out, ref) <= k0_tol(qp)
    s.close()


@pytest.mark.parametrize("n,m1,m2", SIZES)
def test_kf_apply_matches_definition(gpu, n, m1, m2):
    qp = synth.gaussian_qp(2000 + n + m2, n, m1, m2)
    s = make(qp)
    s.factor()
    dvec = synth.log_uniform(5, m2, 1e-3, 1e3)
    p = np.random.default_rng(m2).standard_normal(m2)
    q = s.kf_apply(dvec, p)
    ref = reduced.kf_explicit(qp, dvec) @ p
    assert relerr(q, ref) <= k0_tol(qp)
    assert elemerr(q, ref) <= k0_tol(qp)
    s.close()


@pytest.mark.parametrize("prec", [PL, PH, PN])
@pytest.mark.parametrize("n,m1,m2", [(5, 2, 3), (70, 30, 40), (200, 50, 100), (129, 65, 257), (300, 130, 170)])
def test_pcg_matches_direct_reduced_solve(gpu, prec, n, m1, m2):
    qp = synth.gaussian_qp(3000 + n, n, m1, m2)
    s = make(qp)
    s.factor()
    dvec = synth.log_uniform(9, m2, 1e-2, 1e2)
    rhs = np.random.default_rng(3).standard_normal(m2)
    dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=1e-12)
    ref = sla.cho_solve(sla.cho_factor(reduced.kf_explicit(qp, dvec)), rhs)
    assert relerr(dnu, ref) <= 1e-8
    assert info.rel_res <= 1e-11
    s.close()


@pytest.mark.parametrize("n,m1,m2,prec,bound", [(60, 52, 80, PL, 8), (60, 4, 80, PH, 4), (100, 1, 120, PH, 1)])
def test_pcg_iteration_count_follows_the_corollaries(gpu, n, m1, m2, prec, bound):
    qp = synth.gaussian_qp(4000 + m1, n, m1, m2)
    s = make(qp)
    s.factor()
    dvec = synth.log_uniform(2, m2, 1e-2, 1e2)
    rhs = np.random.default_rng(5).standard_normal(m2)
    K = reduced.kf_explicit(qp, dvec)
    P = reduced.P_L(dvec) if prec == PL else reduced.P_H(qp, dvec)
    cf = sla.cho_factor(P)
    _, k_or, _ = reduced.pcg(lambda v: K @ v, rhs, lambda r: sla.cho_solve(cf, r), 1e-6, 10 * m2)
    dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=1e-6)
    # the same CG recurrence in the same precision: same step count up to one
    assert abs(info.iters - k_or) <= 1
    ref = sla.cho_solve(sla.cho_factor(K), rhs)
    assert relerr(dnu, ref) <= 1e-4
    # Corollaries cor:cg1 / cor:cg2: after bound + 1 steps the true residual has
    # collapsed (to rounding level in exact-arithmetic terms; 1e-4 allows the
    # float64 loss of orthogonality seen on the oracle for these instances)
    dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=0.0, maxit=bound + 1, accept=(qpgpu.QP_OK, qpgpu.QP_E_NOCONV))
    assert info.iters == bound + 1
    assert info.rel_res <= 1e-4
    s.close()


def _check_reported(qp, x, lam, nu, info):
    """The KKT score and objective the library reports for its returned iterate
    (computed in float64 on the GPU) agree with the oracle's on the same iterate."""
    sc, _ = kkt.rel_kkt(qp, x, lam, nu)
    assert abs(info.rel_kkt - sc) <= 1e-12 + 1e-6 * sc, (info.rel_kkt, sc)
    f = kkt.objective(qp, x)
    assert abs(info.obj - f) <= 1e-10 * max(1.0, abs(f)), (info.obj, f)


def _check_ipm(qp, x, lam, nu, f_ref):
    sc, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert sc <= 1e-8, parts
    f = kkt.objective(qp, x)
    assert abs(f - f_ref) <= 1e-7 * max(1.0, abs(f_ref))


@pytest.mark.parametrize("prec", [PL, PH])
@pytest.mark.parametrize("seed", list(range(16)))
def test_ipm_small_workload_matches_oracle(gpu, seed, prec):
    qp = synth.gaussian_qp(seed, 200, 50, 100)
    ref = ipm.solve(qp)
    assert ref.converged
    s = make(qp, prec=prec)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    _check_ipm(qp, x, lam, nu, ref.obj)
    _check_reported(qp, x, lam, nu, info)
    assert np.all(nu > 0) and np.all(sl > 0)
    assert info.ipm_iters <= ref.iters + 5
    s.close()


@pytest.mark.parametrize("seed,n,m1,m2", [(0, 5, 2, 8), (1, 4, 1, 6), (2, 6, 3, 10), (3, 3, 1, 5)])
def test_ipm_tiny_matches_active_set_enumeration(gpu, seed, n, m1, m2):
    qp = synth.tiny_qp(seed, n, m1, m2)
    xb, lb, nb, W = bruteforce.solve(qp)
    s = make(qp, prec=qpgpu.QP_PREC_AUTO)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    assert np.max(np.abs(x - xb)) <= 1e-6 * (1 + np.max(np.abs(xb)))
    _check_ipm(qp, x, lam, nu, kkt.objective(qp, xb))
    s.close()


@pytest.mark.parametrize("prec", [PL, PH])
def test_ipm_box_qp_matches_closed_form(gpu, prec):
    qp = synth.box_qp(1, 40, 8)
    xc, lc, nc = boxqp.solve(qp)
    s = make(qp, prec=prec)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    assert np.max(np.abs(x - xc)) <= 1e-6
    assert np.max(np.abs(lam - lc)) <= 1e-6
    _check_ipm(qp, x, lam, nu, kkt.objective(qp, xc))
    s.close()


def test_failure_paths(gpu):
    qp = synth.gaussian_qp(1, 20, 5, 10)
    # solve before factor
    s = make(qp)
    dvec = np.ones(10)
    rhs = np.ones(10)
    dnu = np.empty(10)
    st, _ = qpgpu.qp_pcg_solve(s.ctx, dvec, rhs, dnu, PL, 1e-8, 0)
    assert st == qpgpu.QP_E_STATE
    s.factor()
    # iteration cap
    dv = synth.log_uniform(1, 10, 1e-4, 1e4)
    st, info = qpgpu.qp_pcg_solve(s.ctx, dv, rhs, dnu, PN, 1e-15, 2)
    assert st == qpgpu.QP_E_NOCONV and info.iters == 2
    # non-positive D is rejected
    st, _ = qpgpu.qp_pcg_solve(s.ctx, -dvec, rhs, dnu, PL, 1e-8, 0)
    assert st == qpgpu.QP_E_INVALID
    s.close()
    # H not positive definite
    bad = synth.gaussian_qp(2, 20, 5, 10)
    bad.H = np.ascontiguousarray(-np.eye(20))
    s = make(bad)
    assert qpgpu.qp_factor_K0(s.ctx) == qpgpu.QP_E_NOT_SPD
    s.close()
    # A rank deficient
    bad = synth.gaussian_qp(3, 20, 5, 10)
    bad.A = np.ascontiguousarray(np.vstack([bad.A[:4], bad.A[:1]]))
    s = make(bad)
    assert qpgpu.qp_factor_K0(s.ctx) == qpgpu.QP_E_RANK
    s.close()


def test_device_pointer_path(gpu):
    import torch
    qp = synth.gaussian_qp(5, 70, 30, 40)
    dev = [torch.from_numpy(a).cuda() for a in qp.arrays()]
    s = qpgpu.Solver(*dev, stream=torch.cuda.current_stream().cuda_stream)
    s.factor()
    rhs = torch.from_numpy(np.random.default_rng(0).standard_normal(100)).cuda()
    out = torch.empty_like(rhs)
    assert qpgpu.qp_k0_solve(s.ctx, rhs, out) == qpgpu.QP_OK
    ref = reduced.k0_solve(qp, rhs.cpu().numpy())
    assert relerr(out.cpu().numpy(), ref) <= 1e-10
    s.close()


# --- mixed precision (float32 CG inside float64 refinement) ------------------
@pytest.mark.parametrize("prec", [PL, PH])
@pytest.mark.parametrize("n,m1,m2", [(70, 30, 40), (200, 50, 100), (300, 130, 170)])
def test_mixed_pcg_matches_direct_reduced_solve(gpu, prec, n, m1, m2):
    qp = synth.gaussian_qp(5000 + n, n, m1, m2)
    s = make(qp, precision=qpgpu.QP_MIXED)
    s.factor()
    dvec = synth.log_uniform(9, m2, 1e-2, 1e2)
    rhs = np.random.default_rng(3).standard_normal(m2)
    dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=1e-10)
    ref = sla.cho_solve(sla.cho_factor(reduced.kf_explicit(qp, dvec)), rhs)
    # the refinement drives the float64 residual to rtol; cond(K_F) <= ~1e4 here
    assert info.rel_res <= 1e-10
    assert relerr(dnu, ref) <= 1e-6
    assert info.refinements >= 1
    s.close()


@pytest.mark.parametrize("prec", [PL, PH])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_mixed_ipm_small_workload_matches_oracle(gpu, seed, prec):
    qp = synth.gaussian_qp(seed, 200, 50, 100)
    ref = ipm.solve(qp)
    s = make(qp, prec=prec, precision=qpgpu.QP_MIXED)
    s.factor()
    x, lam, nu, sl, info = s.ipm()
    _check_ipm(qp, x, lam, nu, ref.obj)
    assert info.refinements_total >= 2 * info.ipm_iters
    s.close()

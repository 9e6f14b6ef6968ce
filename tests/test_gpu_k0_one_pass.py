"""Parity of the one-pass K0 product of the CG step against the oracle (needs an MI355X).

For n <= 4096 the implicit CG step forms K0^{-1}_{11} C^T p = M^T Sigma M C^T p
(K0^{-1} = L^{-T} Sigma L^{-1}, M = L^{-1}[:, :n], Sec. 4.1) in a single sweep of
M: each row's v_i = sigma_i M_i u is used at once for M_i^T v_i, and the
per-workgroup partials of w are summed in a fixed order.  qp_kf_apply (float64)
runs that path, so K_F p is compared with the oracle's K_F, at the bar of the
other K_F tests: normwise relative error <= max(1e-10, 100 eps cond(K0)).

Sizes cover every register-row width of the sweep (n up to 512, 1024, 2048 and
4096 doubles per row), odd and even n (the middle row of the folded triangle),
m1 << n and m1 ~ n, and n = 4097 where the library keeps the two sweeps.
"""
import numpy as np
import pytest

import synth
from oracle import reduced
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu

SIZES = [(1, 1, 1), (2, 1, 1), (3, 2, 5), (64, 63, 10), (129, 65, 40), (511, 7, 33), (513, 300, 64),
         (1023, 1, 17), (1025, 512, 100), (2047, 100, 200), (2049, 2049, 31), (4095, 9, 64), (4096, 64, 257)]


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def k0_tol(qp):
    return max(1e-10, 100 * np.finfo(float).eps * np.linalg.cond(reduced.K0_matrix(qp)))


@pytest.mark.parametrize("n,m1,m2", SIZES)
def test_one_pass_kf_apply_matches_oracle(gpu, n, m1, m2):
    qp = synth.gaussian_qp(4400 + n + m1, n, m1, m2)
    s = qpgpu.Solver(*qp.arrays())
    assert s.k0_one_pass()
    s.factor()
    dvec = synth.log_uniform(11, m2, 1e-3, 1e3)
    p = np.random.default_rng(n + m2).standard_normal(m2)
    q = s.kf_apply(dvec, p)
    ref = reduced.kf_apply(qp, dvec, p)
    assert relerr(q, ref) <= k0_tol(qp)
    assert np.max(np.abs(q - ref)) <= k0_tol(qp) * np.max(np.abs(ref))  # element by element
    # fixed summation order: a second product is bitwise the same
    assert np.array_equal(q, s.kf_apply(dvec, p))
    s.close()


def test_two_sweeps_above_the_one_pass_limit(gpu):
    qp = synth.gaussian_qp(4497, 4097, 3, 8)
    s = qpgpu.Solver(*qp.arrays())
    assert not s.k0_one_pass()
    s.factor()
    dvec = synth.log_uniform(12, 8, 1e-3, 1e3)
    p = np.random.default_rng(5).standard_normal(8)
    assert relerr(s.kf_apply(dvec, p), reduced.kf_apply(qp, dvec, p)) <= k0_tol(qp)
    s.close()


def test_explicit_form_keeps_its_own_operator(gpu):
    qp = synth.gaussian_qp(4498, 100, 20, 30)
    s = qpgpu.Solver(*qp.arrays(), kf_form=qpgpu.QP_KF_EXPLICIT)
    assert not s.k0_one_pass()
    s.close()


@pytest.mark.parametrize("prec", [qpgpu.QP_PREC_LOW_DOF, qpgpu.QP_PREC_FEW_EQ])
def test_one_pass_pcg_at_width_8(gpu, prec):
    """A PCG solve whose every step runs the widest register rows (n = 4000)."""
    import scipy.linalg as sla
    qp = synth.gaussian_qp(4499, 4000, 200, 96)
    s = qpgpu.Solver(*qp.arrays())
    s.factor()
    dvec = synth.log_uniform(13, 96, 1e-2, 1e2)
    rhs = np.random.default_rng(7).standard_normal(96)
    dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=1e-12)
    ref = sla.cho_solve(sla.cho_factor(reduced.kf_explicit(qp, dvec)), rhs)
    assert relerr(dnu, ref) <= 1e-8
    assert info.rel_res <= 1e-11
    s.close()

"""qp_factor_K0_static, the factorization entry point that allocates no device
memory (its set-up scratch lives in a fixed device array), against qp_factor_K0
through the C ABI (needs an MI355X).

Both run the same kernels in the same launch shapes; only the addresses of the
scratch buffers differ, so the stored factor -- and every solve made with it --
is bitwise the same.  Two calls in a row share the GPU's array, the second with
a smaller QP; a QP whose scratch exceeds the array is refused and leaves the
context usable.
"""
import numpy as np
import pytest

import synth
from oracle import kkt
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu

PL, PH = qpgpu.QP_PREC_LOW_DOF, qpgpu.QP_PREC_FEW_EQ


def _run(qp, static, prec, kf_form=qpgpu.QP_KF_IMPLICIT):
    s = qpgpu.Solver(*qp.arrays(), prec=prec, kf_form=kf_form)
    s.factor(static=static)
    rhs = np.random.default_rng(qp.n).standard_normal(qp.n + qp.m1)
    k0 = s.k0_solve(rhs)
    x, lam, nu, sl, info = s.ipm()
    s.close()
    return (k0, x, lam, nu, sl), info


@pytest.mark.parametrize("prec,kf_form", [(PH, qpgpu.QP_KF_IMPLICIT), (PL, qpgpu.QP_KF_IMPLICIT),
                                          (PH, qpgpu.QP_KF_EXPLICIT)])
def test_static_factor_equals_allocating_factor(gpu, prec, kf_form):
    # the second call, with a smaller QP, finds what the first left in the array
    for seed, n, m1, m2 in [(31, 900, 225, 450), (32, 200, 50, 100)]:
        print(f"no-alloc factor: seed {seed} n={n} m1={m1} m2={m2} prec={prec} kf={kf_form}", flush=True)
        qp = synth.gaussian_qp(seed, n, m1, m2)
        ref, ref_info = _run(qp, False, prec, kf_form)
        got, info = _run(qp, True, prec, kf_form)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        assert (info.ipm_iters, info.pcg_iters_total) == (ref_info.ipm_iters, ref_info.pcg_iters_total)
        score, parts = kkt.rel_kkt(qp, got[1], got[2], got[3])
        assert score <= 1e-8, parts


def test_static_factor_refuses_a_qp_beyond_the_array(gpu):
    qp = synth.gaussian_qp(33, 2048, 512, 1024)  # P_H scratch of about 95 MB
    s = qpgpu.Solver(*qp.arrays(), prec=PH)
    st = qpgpu.qp_factor_K0_static(s.ctx)
    assert st == qpgpu.QP_E_INVALID
    assert "scratch" in qpgpu.qp_last_error(s.ctx)
    # nothing was run: the context factors normally afterwards
    s.factor()
    rhs = np.random.default_rng(5).standard_normal(qp.n + qp.m1)
    out = s.k0_solve(rhs)
    assert np.all(np.isfinite(out))
    s.close()
    # and the array still serves a QP that fits
    small = synth.gaussian_qp(34, 300, 75, 150)
    a, ia = _run(small, True, PH)
    b, ib = _run(small, False, PH)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)

"""Graph replay of the CG poll chunks (options.cg_graph) against plain launches
(needs an MI355X).

The captured chunk holds the same kernels with the same arguments as the chunk
launched step by step, so every result is bitwise the same; each replay is
preceded by the library's own eager work (right-hand sides, refinement,
recovery) and a host poll, which exercises replays after the first.
"""
import numpy as np
import pytest

import synth
from oracle import ipm, kkt
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [qpgpu.QP_PREC_LOW_DOF, qpgpu.QP_PREC_FEW_EQ])
@pytest.mark.parametrize("precision", [qpgpu.QP_FP64, qpgpu.QP_MIXED])
def test_graph_replay_is_bitwise_the_launched_chunks(gpu, prec, precision):
    qp = synth.gaussian_qp(3, 200, 50, 100)
    out = []
    for graph in (0, 1):
        s = qpgpu.Solver(*qp.arrays(), prec=prec, precision=precision, cg_graph=graph)
        s.factor()
        out.append(s.ipm())
        # a standalone PCG solve after the IPM reuses or re-captures the chunk for its buffers
        rhs = np.random.default_rng(4).standard_normal(qp.m2)
        dvec = np.random.default_rng(5).uniform(0.1, 10.0, qp.m2)
        out[-1] = out[-1] + s.pcg(dvec, rhs, prec=prec, rtol=1e-10)
        s.close()
    (x0, l0, n0, s0, i0, d0, p0), (x1, l1, n1, s1, i1, d1, p1) = out
    for a, b in ((x0, x1), (l0, l1), (n0, n1), (s0, s1), (d0, d1)):
        assert np.array_equal(a, b)
    assert (i0.ipm_iters, i0.pcg_iters_total) == (i1.ipm_iters, i1.pcg_iters_total)
    assert p0.iters == p1.iters
    ref = ipm.solve(qp)
    score, parts = kkt.rel_kkt(qp, x1, l1, n1)
    assert score <= 1e-8, parts
    assert abs(kkt.objective(qp, x1) - ref.obj) <= 1e-7 * max(1.0, abs(ref.obj))

"""Batches at the sizes of the batched and streamed workloads (needs an MI355X).

* A 24-QP sample of the 512-QP draw (synth.batch_sample: its 8 largest QPs,
  n >= 1008, and 16 spread over n = 64..1020), solved as one batch in mixed
  precision and in float64.
* Batches whose largest QP is bigger than the 512-QP draw allows
  (synth.large_batch_sizes: n = 1500, 2500, 4000 with m1 = n/4, m2 = n/2) next
  to small ones.  A batched launch of the one-pass K0 sweep keeps every QP's
  row of M in registers at the width of the largest QP in its list, 512
  float64 (1024 float32) columns per step of the width: n = 1500 runs the
  float32 sweep at width 2 and the float64 sweep at width 4, n = 2500 and 4000
  the float32 sweep at width 4 and the float64 sweep at width 8 -- widths the
  n <= 1024 draw never reaches.

Every result is checked against the oracle: its relative KKT score of the
returned iterate <= 1e-8 (oracle.kkt on the host) and the objective within
1e-7 * max(1, |f*|) of the oracle's full-KKT IPM, read from the golden files
tests/golden/oracle_set_*.json that tests/golden/make_golden.py writes with the
oracle alone.  The score the library reports must agree with the oracle's.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import kkt
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
AUTO = qpgpu.QP_PREC_AUTO


def golden_set(name):
    with open(os.path.join(HERE, "golden", f"oracle_set_{name}.json")) as f:
        return {r["seed"]: r for r in json.load(f)["records"]}


@pytest.fixture(scope="module")
def goldens():
    g = golden_set("batch24")
    g.update(golden_set("large"))
    return g


def run_batch(qps, precision):
    b = qpgpu.Batch(0, prec=AUTO, precision=precision)
    tickets = [b.admit(*qp.arrays()) for qp in qps]
    assert all(t is not None for t in tickets)
    b.step(100000)
    assert set(b.finished()) == set(tickets)
    out = [b.collect(t) for t in tickets]
    assert b.query()["bytes_used"] == 0
    b.close()
    return out


def check(qp, seed, res, goldens):
    x, lam, nu, s, info = res
    g = goldens[seed]
    assert g["converged"] and (g["n"], g["m1"], g["m2"]) == (qp.n, qp.m1, qp.m2)
    score, parts = kkt.rel_kkt(qp, x, lam, nu)
    assert score <= 1e-8, (seed, parts)
    f = kkt.objective(qp, x)
    assert abs(f - g["obj"]) <= 1e-7 * max(1.0, abs(g["obj"])), (seed, f, g["obj"])
    assert abs(info.rel_kkt - score) <= 1e-12 + 1e-6 * score, (seed, info.rel_kkt, score)
    assert abs(info.obj - f) <= 1e-10 * max(1.0, abs(f))
    assert np.all(nu > 0) and np.all(s > 0)
    assert info.status == qpgpu.QP_OK and info.ipm_iters <= g["iters"] + 10
    return info


@pytest.mark.parametrize("precision", [qpgpu.QP_MIXED, qpgpu.QP_FP64])
def test_batch_sample_of_the_512_qp_draw(gpu, goldens, precision):
    specs = synth.batch_sample()
    assert len(specs) == 24 and max(sp[1] for sp in specs) >= 1008
    qps = [synth.gaussian_qp(*sp) for sp in specs]
    res = run_batch(qps, precision)
    fallbacks = refin = 0
    for sp, qp, r in zip(specs, qps, res):
        info = check(qp, sp[0], r, goldens)
        fallbacks += info.fp64_fallbacks
        refin += info.refinements_total
    if precision == qpgpu.QP_MIXED:
        assert refin > 0  # the float32 inner solves ran inside float64 refinement
    else:
        assert refin == 0 and fallbacks == 0


LARGE = {sp[1]: sp for sp in synth.large_batch_sizes()}


@pytest.mark.parametrize("precision", [qpgpu.QP_MIXED, qpgpu.QP_FP64])
@pytest.mark.parametrize("large_n", [[1500], [2500, 4000]])
def test_batch_with_qps_beyond_the_draw(gpu, goldens, precision, large_n):
    small = [sp for sp in synth.batch_sample() if sp[1] <= 400][:3]
    specs = [LARGE[n] for n in large_n] + small
    qps = [synth.gaussian_qp(*sp) for sp in specs]
    res = run_batch(qps, precision)
    for sp, qp, r in zip(specs, qps, res):
        check(qp, sp[0], r, goldens)


def test_large_qp_alone_equals_in_mix(gpu):
    """The n = 1500 QP batched with small ones gives the bits it gives alone,
    although the mix launches at the width the largest QP needs."""
    small = [sp for sp in synth.batch_sample() if sp[1] <= 400][:3]
    qps = [synth.gaussian_qp(*sp) for sp in small] + [synth.gaussian_qp(*LARGE[1500])]
    mix = run_batch(qps, qpgpu.QP_MIXED)
    for qp, (x, lam, nu, s, info) in zip(qps, mix):
        (xa, la, na, sa, ia), = run_batch([qp], qpgpu.QP_MIXED)
        assert np.array_equal(x, xa) and np.array_equal(nu, na) and np.array_equal(lam, la)
        assert info.pcg_iters_total == ia.pcg_iters_total

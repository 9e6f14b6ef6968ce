"""Serving: continuous batching of a stream of QPs (needs an MI355X).

A seeded trace of 24 requests of the streamed workload's mix (n log-uniform in
128..4096, up to n = 4052 here; m1 = n U(1/8, 1/2), m2 = n U(1/2, 1)) arrives
as a Poisson stream at a server whose device arena holds about a third of the
trace at once, so admission waits for memory and requests that arrive while
others run join the batch in flight.  For every request: the oracle's relative
KKT score of the returned iterate is <= 1e-8, and the iterate is bitwise the one
the same QP gives alone (each QP's launch shapes and arithmetic depend only on
that QP).  The latency accounting is checked for consistency.
"""
import numpy as np
import pytest

import synth
from oracle import kkt
from paper_2104_12916_amd import qpgpu, serve

pytestmark = pytest.mark.gpu

OPTS = dict(prec=qpgpu.QP_PREC_AUTO, precision=qpgpu.QP_MIXED)


@pytest.fixture(scope="module")
def trace():
    specs = synth.serving_stream(24, seed=5000)
    return specs, [synth.gaussian_qp(*sp) for sp in specs]


def test_serving_trace_matches_oracle_and_solo_runs(gpu, trace):
    specs, qps = trace
    assert max(sp[1] for sp in specs) >= 4000
    opt = qpgpu.qp_default_options(**OPTS)
    fps = [qpgpu.qp_batch_footprint(opt, qp.n, qp.m1, qp.m2) for qp in qps]
    budget = max(max(fps), sum(fps) // 3)
    arrivals = serve.poisson_arrivals(len(qps), rate=40.0, seed=5001)
    with serve.Server(budget, **OPTS) as srv:
        res = srv.run([qp.arrays() for qp in qps], arrivals)
        st = srv.stats
    assert st.memory_waits > 0              # the memory cap bound admission
    assert st.peak_in_flight >= 3           # requests overlapped on the device
    assert st.peak_bytes_used <= budget
    for k, (qp, r) in enumerate(zip(qps, res)):
        assert r.rid == k and r.status == qpgpu.QP_OK
        assert r.arrival <= r.admitted <= r.finished and r.latency > 0
        score, parts = kkt.rel_kkt(qp, r.x, r.lam, r.nu)
        assert score <= 1e-8, (k, specs[k], parts)
        assert abs(r.info.rel_kkt - score) <= 1e-12 + 1e-6 * score
    summ = serve.latency_summary(res)
    assert summ["count"] == 24 and 0 < summ["p50_ms"] <= summ["p99_ms"] <= summ["max_ms"]
    # every request alone (in an arena of its own footprint) gives the same bits
    for k, qp in enumerate(qps):
        with serve.Server(fps[k], **OPTS) as solo:
            (a,) = solo.run([qp.arrays()])
        r = res[k]
        assert np.array_equal(a.x, r.x) and np.array_equal(a.lam, r.lam), k
        assert np.array_equal(a.nu, r.nu) and np.array_equal(a.s, r.s), k
        assert a.info.pcg_iters_total == r.info.pcg_iters_total and a.info.ipm_iters == r.info.ipm_iters


def test_request_larger_than_the_arena_is_refused(gpu):
    qp = synth.gaussian_qp(1, 300, 60, 150)
    with serve.Server(1 << 20, **OPTS) as srv:   # 1 MiB: far too small
        with pytest.raises(ValueError, match="more than the arena"):
            srv.submit(*qp.arrays())
        assert not srv.busy


@pytest.mark.parametrize("side_stream", [False, True])
def test_device_inputs_written_on_torch_stream_just_before_the_call(gpu, side_stream):
    """Inputs that torch is still writing when the call is made are read after torch's work."""
    import torch
    qp = synth.gaussian_qp(9, 300, 80, 150)
    ref = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_FEW_EQ)
    ref.factor()
    xr, lr, nr, sr, _ = ref.ipm()
    ref.close()
    staged = [torch.from_numpy(a).cuda() for a in qp.arrays()]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream() if side_stream else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        dev = [torch.zeros_like(t) for t in staged]
        big = torch.rand(3072, 3072, dtype=torch.float64, device="cuda")
        for _ in range(6):                         # keep the stream busy for a few ms
            big = (big @ big) * (1.0 / 3072)
        for t, src in zip(dev, staged):
            t.copy_(src)                          # written on the stream after the matmuls
        s = qpgpu.Solver(*dev, prec=qpgpu.QP_PREC_FEW_EQ)   # stream=None: ordered after torch's work
        s.factor()
        x, lam, nu, sl, info = s.ipm()
        s.close()
        b = qpgpu.Batch(0, prec=qpgpu.QP_PREC_FEW_EQ)
        for t in dev:
            t.zero_()
        for _ in range(6):
            big = (big @ big) * (1.0 / 3072)
        for t, src in zip(dev, staged):
            t.copy_(src)
        tk = b.admit(*dev)
        b.step(10000)
        xb, lb, nb, sb, ib = b.collect(tk)
        b.close()
    assert np.array_equal(x, xr) and np.array_equal(nu, nr)
    score, parts = kkt.rel_kkt(qp, xb, lb, nb)
    assert score <= 1e-8, parts

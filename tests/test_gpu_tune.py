"""Parity of the CG step under every launch shape the tune table can select (needs an MI355X).

The launch-shape table changes only how the streaming kernels split and load
their work (workgroups per CU, loads in flight, one-pass sweep width, update
width, cache policy), never what they compute, so K_F p and the PCG solution
must match the oracle at the usual bars whichever entry a call selects.  Calls
on one QP select the bucket of its n; the test sets a table whose base entry and
bucket entries differ in every kernel key and checks QPs on both sides of the
bucket edge, plus the cache file the autotuner writes.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import reduced
from paper_2104_12916_amd import qpgpu

pytestmark = pytest.mark.gpu

SHAPES = [
    "rows_bpc=1,rows_unroll=4,sym_wg=1,sym_rows=2,ld_nt=0,upd_threads=256,cols_bpc=1,cols_unroll=4",
    "rows_bpc=8,rows_unroll=8,sym_wg=4,sym_rows=4,ld_nt=3,upd_threads=1024,cols_bpc=4,cols_unroll=8",
    "rows_bpc=6,rows_unroll=4,sym_wg=3,sym_rows=2,ld_nt=2,upd_threads=512,qe_stage=1,rows_stage=1",
]


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def k0_tol(qp):
    return max(1e-10, 100 * np.finfo(float).eps * np.linalg.cond(reduced.K0_matrix(qp)))


@pytest.fixture
def table():
    before = qpgpu.tune_get()
    yield before
    qpgpu.tune_set(before)


def check_qp(qp, seed):
    s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_LOW_DOF)
    s.factor()
    dvec = synth.log_uniform(seed, qp.m2, 1e-3, 1e3)
    p = np.random.default_rng(seed).standard_normal(qp.m2)
    assert relerr(s.kf_apply(dvec, p), reduced.kf_apply(qp, dvec, p)) <= k0_tol(qp)
    pcg_matches(s, qp, seed, qpgpu.QP_PREC_LOW_DOF)
    s.close()


def pcg_matches(s, qp, seed, prec):
    dvec = synth.log_uniform(seed + 2, qp.m2, 1e-2, 1e2)
    rhs = np.random.default_rng(seed + 1).standard_normal(qp.m2)
    dnu, info = s.pcg(dvec, rhs, prec=prec, rtol=1e-12)
    ref = sla.cho_solve(sla.cho_factor(reduced.kf_explicit(qp, dvec)), rhs)
    assert relerr(dnu, ref) <= 1e-8
    assert info.rel_res <= 1e-11


@pytest.mark.parametrize("shape", range(len(SHAPES)))
@pytest.mark.parametrize("n,m1,m2", [(300, 200, 150), (700, 500, 333)])
def test_bucket_and_base_shapes_match_oracle(gpu, table, shape, n, m1, m2):
    other = SHAPES[(shape + 1) % len(SHAPES)]
    base = table.splitlines()[0]
    # base entry with one shape, bucket n <= 512 with another: n = 300 runs the bucket, n = 700 the base
    qpgpu.tune_set(f"{base}\ndefault {other}\nn<=512 {SHAPES[shape]}")
    check_qp(synth.gaussian_qp(5100 + n + shape, n, m1, m2), 40 + shape)


def test_few_eq_path_and_nested_buckets(gpu, table):
    base = table.splitlines()[0]
    qpgpu.tune_set(f"{base}\nn<=256 {SHAPES[1]}\nn<=1024 {SHAPES[0]}")
    qp = synth.gaussian_qp(5301, 200, 20, 120)
    s = qpgpu.Solver(*qp.arrays(), prec=qpgpu.QP_PREC_FEW_EQ)
    s.factor()
    pcg_matches(s, qp, 7, qpgpu.QP_PREC_FEW_EQ)
    s.close()
    check_qp(synth.gaussian_qp(5302, 1000, 700, 400), 9)


def test_autotune_cache_is_loaded(gpu, table):
    path = os.path.join(os.path.dirname(os.path.abspath(qpgpu.LIB_PATH)), "autotune_gfx950.txt")
    if "QPGPU_TUNE" in os.environ or "QPGPU_AUTOTUNE_CACHE" in os.environ or not os.path.exists(path):
        pytest.skip("no autotune cache in use")
    with open(path) as f:
        lines = [ln.strip() for ln in f if ln.strip().startswith("n<=")]
    loaded = [ln for ln in table.splitlines() if ln.startswith("n<=")]
    assert [ln.split()[0] for ln in loaded] == [ln.split()[0] for ln in lines]
    for got, want in zip(loaded, lines):
        kv = dict(x.split("=") for x in got.split()[1].split(","))
        for x in want.split()[1].split(","):
            k, v = x.split("=")
            assert kv[k] == v, (got, want)


ONE_PASS_SIZES = [(1, 1, 1), (3, 2, 5), (129, 65, 40), (513, 300, 64), (1025, 512, 100), (2049, 2049, 31),
                  (4095, 9, 64), (4096, 3072, 257)]


@pytest.mark.parametrize("sym_wg", [1, 2])
@pytest.mark.parametrize("n,m1,m2", ONE_PASS_SIZES)
def test_pipelined_one_pass_is_bitwise_the_two_row_sweep(gpu, table, sym_wg, n, m1, m2):
    """The pipelined one-pass sweep reads the same rows in the same order with the
    same arithmetic as the two-rows-per-round sweep of one-team workgroups: K_F p
    is bitwise equal."""
    base = table.splitlines()[0]
    qp = synth.gaussian_qp(5500 + n + m1, n, m1, m2)
    s = qpgpu.Solver(*qp.arrays())
    assert s.k0_one_pass()
    s.factor()
    dvec = synth.log_uniform(13, m2, 1e-3, 1e3)
    p = np.random.default_rng(n + 7).standard_normal(m2)
    out = {}
    for pipe in (0, 1):
        for nt in (1, 3):
            qpgpu.tune_set(f"{base}\ndefault sym_rows=2,sym_pipe={pipe},sym_wg={sym_wg},ld_nt={nt},sym_teams=1")
            out[pipe, nt] = s.kf_apply(dvec, p)
    s.close()
    assert relerr(out[1, 1], reduced.kf_apply(qp, dvec, p)) <= k0_tol(qp)
    for key in out:
        assert np.array_equal(out[key], out[0, 1]), key


TEAM_SIZES = [(1025, 512, 100), (2049, 2049, 31), (1500, 700, 64), (4096, 3072, 257)]


@pytest.mark.parametrize("sym_wg", [2, 4])
@pytest.mark.parametrize("n,m1,m2", TEAM_SIZES)
def test_two_team_one_pass_matches_one_team(gpu, table, sym_wg, n, m1, m2):
    """Workgroups of two teams (each with its own rows and partial, added in team
    order before the one partial is written) give the K_F product of the
    one-team sweep up to the order of the additions, and the oracle's.  With
    sym_units=1 every size here has enough units for two teams per CU."""
    base = table.splitlines()[0]
    qp = synth.gaussian_qp(5700 + n + m1, n, m1, m2)
    s = qpgpu.Solver(*qp.arrays())
    assert s.k0_one_pass()
    s.factor()
    dvec = synth.log_uniform(17, m2, 1e-3, 1e3)
    p = np.random.default_rng(n + 11).standard_normal(m2)
    out = {}
    for teams in (1, 2):
        for rows in (2, 4):
            qpgpu.tune_set(f"{base}\ndefault sym_pipe=0,sym_units=1,sym_wg={sym_wg},sym_rows={rows},"
                           f"sym_teams={teams}")
            out[teams, rows] = s.kf_apply(dvec, p)
    s.close()
    ref = reduced.kf_apply(qp, dvec, p)
    tol = k0_tol(qp)
    for key, v in out.items():
        assert relerr(v, ref) <= tol, key
        assert relerr(v, out[1, 4]) <= tol, key


def test_pipelined_one_pass_in_batches(gpu, table):
    """Batched one-pass sweep (every QP of the batch in one launch) with and
    without pipelining: bitwise the same IPM results."""
    base = table.splitlines()[0]
    rng = np.random.default_rng(77)
    qps = [synth.gaussian_qp(5600 + i, int(nn), int(nn) // 4, int(nn) // 2)
           for i, nn in enumerate(rng.integers(40, 700, size=6))]
    res = {}
    for pipe in (0, 1):
        qpgpu.tune_set(f"{base}\ndefault sym_rows=2,sym_pipe={pipe}")
        b = qpgpu.Batch(0, prec=qpgpu.QP_PREC_FEW_EQ)
        tickets = [b.admit(*qp.arrays()) for qp in qps]
        b.step(1000)
        assert set(b.finished()) == set(tickets)
        res[pipe] = [b.collect(t)[0] for t in tickets]
        b.close()
    for x0, x1, qp in zip(res[0], res[1], qps):
        assert np.array_equal(x0, x1)


def test_hbm_read_probe_rate_is_plausible(gpu):
    """The read-rate probe streams its buffer: a rate between 1 TB/s and the 8 TB/s
    interface peak (a 1 GiB buffer, 4x the last-level cache)."""
    nbytes = 1 << 30
    gbs = nbytes / (qpgpu.hbm_read_time(nbytes, 8, 5) * 1e-3) / 1e9
    assert 1000.0 < gbs < 8000.0, gbs

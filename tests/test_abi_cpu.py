"""The C-ABI library loads and exports every symbol declared in include/qpgpu.h.

No compute call is made here (no GPU): only symbol lookup, static strings,
option defaults and argument validation that returns before touching a device.
"""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2104_12916_amd import qpgpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "qpgpu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_[a-zA-Z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = qpgpu.lib()
    names = header_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(qpgpu.EXPORTS)


def test_status_strings_and_defaults():
    assert qpgpu.qp_status_str(qpgpu.QP_OK) == "ok"
    assert "positive definite" in qpgpu.qp_status_str(qpgpu.QP_E_NOT_SPD)
    assert qpgpu.qp_status_str(99) == "unknown status"
    o = qpgpu.qp_default_options()
    assert o.rtol_kkt == 1e-9 and o.tau == 0.995 and o.max_ipm == 200
    assert o.prec == qpgpu.QP_PREC_AUTO and o.precision == qpgpu.QP_FP64
    assert o.kf_form == qpgpu.QP_KF_IMPLICIT
    assert qpgpu.lib().qp_last_error(None) == b""
    qpgpu.lib().qp_destroy(None)


def _qp(n=6, m1=2, m2=4):
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((n, n))
    H = Q.T @ Q / n + np.eye(n)
    return (np.ascontiguousarray(H), rng.standard_normal(n), rng.standard_normal((m1, n)),
            rng.standard_normal(m1), rng.standard_normal((m2, n)), rng.standard_normal(m2))


@pytest.mark.parametrize("case", ["m1_zero", "m1_gt_n", "m2_zero", "nan", "asym", "bad_tau"])
def test_setup_rejects_invalid_input_before_device_work(case):
    H, c, A, b, C, d = _qp()
    L = qpgpu.lib()
    ctx = ct.c_void_p()
    n, m1, m2 = 6, 2, 4
    opt = qpgpu.qp_default_options()
    if case == "m1_zero":
        m1 = 0
    elif case == "m1_gt_n":
        m1 = 7
    elif case == "m2_zero":
        m2 = 0
    elif case == "nan":
        c = c.copy()
        c[3] = np.nan
    elif case == "asym":
        H = H.copy()
        H[0, 1] += 1e-6
    elif case == "bad_tau":
        opt.tau = 1.5
    ptrs = [a.ctypes.data_as(ct.c_void_p) for a in (H, c, A, b, C, d)]
    st = L.qp_setup(ct.byref(ctx), n, m1, m2, *ptrs, qpgpu.QP_MEM_HOST, ct.byref(opt), None)
    assert st == qpgpu.QP_E_INVALID
    assert not ctx.value


def test_null_context_calls_are_rejected():
    L = qpgpu.lib()
    assert L.qp_factor_K0(None) == qpgpu.QP_E_INVALID
    assert L.qp_factor_K0_static(None) == qpgpu.QP_E_INVALID
    assert L.qp_ipm_solve(None, None, None, None, None, 0, None) == qpgpu.QP_E_INVALID
    assert L.qp_pcg_solve(None, None, None, None, 0, 1, 1e-8, 0, None) == qpgpu.QP_E_INVALID
    assert L.qp_ctx_bytes(None) == 0


def test_static_scratch_size_matches_the_header():
    text = open(os.path.join(ROOT, "include", "qpgpu.h")).read()
    m = re.search(r"#define QPGPU_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == qpgpu.STATIC_SCRATCH_BYTES


def test_binding_marshalling_rejects_wrong_dtypes():
    with pytest.raises(TypeError):
        qpgpu._ptr(np.zeros(3, dtype=np.float32))
    with pytest.raises(TypeError):
        qpgpu._ptr(np.zeros((3, 3))[:, :2])


def test_batch_calls_reject_null_handles():
    L = qpgpu.lib()
    LL = ct.c_longlong(0)
    n_done = ct.c_int(0)
    assert L.qp_batch_create(None, None, 0, None) == qpgpu.QP_E_INVALID
    assert L.qp_batch_admit(None, 3, 1, 2, None, None, None, None, None, None, 0, ct.byref(LL)) == qpgpu.QP_E_INVALID
    assert L.qp_batch_step(None, 1, ct.byref(n_done)) == qpgpu.QP_E_INVALID
    assert L.qp_batch_finished(None, None, 0, ct.byref(n_done)) == qpgpu.QP_E_INVALID
    assert L.qp_batch_collect(None, 1, None, None, None, None, 0, None) == qpgpu.QP_E_INVALID
    assert L.qp_batch_query(None, None, None, None, None, None) == qpgpu.QP_E_INVALID
    assert L.qp_batch_last_error(None) == b""
    L.qp_batch_destroy(None)


def test_batch_footprint_is_positive_monotone_and_validates():
    opt = qpgpu.qp_default_options(prec=qpgpu.QP_PREC_FEW_EQ)
    f = [qpgpu.qp_batch_footprint(opt, n, n // 4, n // 2) for n in (64, 128, 512, 1024)]
    assert all(a > 0 for a in f) and f == sorted(f)
    # the footprint holds at least the matrices H, A, C and the inverse factor of K0
    n = 512
    assert f[2] >= 8 * (n * n + (n // 4) * n + (n // 2) * n + (n + n // 4) ** 2)
    # P_L needs no X_P buffers; the mixed path adds float32 copies
    assert qpgpu.qp_batch_footprint(qpgpu.qp_default_options(prec=qpgpu.QP_PREC_LOW_DOF), 512, 128, 256) < f[2]
    assert qpgpu.qp_batch_footprint(qpgpu.qp_default_options(prec=qpgpu.QP_PREC_FEW_EQ, precision=qpgpu.QP_MIXED),
                                    512, 128, 256) > f[2]
    # the explicit operator holds E (m2 x m2) and, during the factorization, Y (N x m2)
    fe = qpgpu.qp_batch_footprint(qpgpu.qp_default_options(prec=qpgpu.QP_PREC_FEW_EQ,
                                                           kf_form=qpgpu.QP_KF_EXPLICIT), 512, 128, 256)
    assert fe >= 8 * (n * n + 128 * n + 256 * n + 640 ** 2 + 256 * 256 + 640 * 256) and fe != f[2]
    assert qpgpu.qp_batch_footprint(qpgpu.qp_default_options(kf_form=7), 5, 2, 1) == 0
    assert qpgpu.qp_batch_footprint(opt, 0, 1, 1) == 0
    assert qpgpu.qp_batch_footprint(opt, 5, 6, 1) == 0
    assert qpgpu.qp_batch_footprint(qpgpu.qp_default_options(tau=2.0), 5, 2, 1) == 0


def test_query_calls_accept_null():
    L = qpgpu.lib()
    cnt = ct.c_int(7)
    assert L.qp_k0_one_pass(None) == 0
    assert L.qp_c_identity(None) == 0
    assert L.qp_ipm_cg_steps(None, None, None, 0, ct.byref(cnt)) == qpgpu.QP_E_INVALID


def test_ph_form_default_and_validation():
    o = qpgpu.qp_default_options()
    assert o.ph_form == qpgpu.QP_PH_EXACT
    L = qpgpu.lib()
    n, m1, m2 = 4, 2, 3
    arrs = [np.eye(n), np.zeros(n), np.ones((m1, n)), np.zeros(m1), np.ones((m2, n)), np.zeros(m2)]
    ptrs = [a.ctypes.data_as(ct.c_void_p) for a in arrs]
    bad = qpgpu.qp_default_options(ph_form=5)
    ctx = ct.c_void_p()
    assert L.qp_setup(ct.byref(ctx), n, m1, m2, *ptrs, qpgpu.QP_MEM_HOST, ct.byref(bad), None) == qpgpu.QP_E_INVALID
    assert not ctx.value


def test_shared_calls_reject_null_handles_and_unsupported_options():
    L = qpgpu.lib()
    P = ct.c_void_p
    n, m1, m2 = 4, 2, 3
    H, A, C = np.eye(n), np.ones((m1, n)), np.ones((m2, n))
    hp, ap, cp = (a.ctypes.data_as(P) for a in (H, A, C))
    out = P()
    opt = qpgpu.qp_default_options()
    assert L.qp_shared_setup(None, n, m1, m2, hp, ap, cp, qpgpu.QP_MEM_HOST, ct.byref(opt), None) == qpgpu.QP_E_INVALID
    assert L.qp_shared_setup(ct.byref(out), 0, m1, m2, hp, ap, cp, qpgpu.QP_MEM_HOST, ct.byref(opt),
                             None) == qpgpu.QP_E_INVALID
    # options the shared solver does not take, and a non-symmetric H, fail before any device work
    for bad in (dict(precision=qpgpu.QP_MIXED), dict(kf_form=qpgpu.QP_KF_EXPLICIT),
                dict(prec=qpgpu.QP_PREC_FEW_EQ)):
        o = qpgpu.qp_default_options(**bad)
        assert L.qp_shared_setup(ct.byref(out), n, m1, m2, hp, ap, cp, qpgpu.QP_MEM_HOST, ct.byref(o),
                                 None) == qpgpu.QP_E_INVALID
        assert not out.value
    Hn = np.eye(n)
    Hn[0, 1] = 1.0
    assert L.qp_shared_setup(ct.byref(out), n, m1, m2, Hn.ctypes.data_as(P), ap, cp, qpgpu.QP_MEM_HOST,
                             ct.byref(opt), None) == qpgpu.QP_E_INVALID
    assert L.qp_shared_pcg_solve(None, 1, None, None, None, 0, 1, 1e-8, 0, None) == qpgpu.QP_E_INVALID
    assert L.qp_shared_ipm_solve(None, 1, None, None, None, None, None, None, None, 0, None) == qpgpu.QP_E_INVALID
    assert L.qp_shared_last_error(None) == b""
    L.qp_shared_destroy(None)


def test_tune_table_set_get_and_validation():
    before = qpgpu.tune_get()
    assert before.startswith("default ")
    try:
        qpgpu.tune_set("# comment\narch gfx950\ndefault rows_bpc=2\nn<=512 sym_wg=1,upd_threads=256\nn<=256 sym_rows=2")
        t = qpgpu.tune_get().splitlines()
        assert t[0].startswith("default ") and "rows_bpc=2" in t[0]
        assert t[1].startswith("n<=256 ") and "sym_rows=2" in t[1] and "rows_bpc=2" in t[1]  # buckets sorted
        assert t[2].startswith("n<=512 ") and "sym_wg=1" in t[2] and "upd_threads=256" in t[2]
        # the keys of the two-team one-pass sweep, the wavefront-row batched sweep and the fold bits
        qpgpu.tune_set("default sym_teams=1,bsym_wave=0,cg_fold=7\nn<=512 sym_teams=2,cg_fold=0")
        t = qpgpu.tune_get().splitlines()
        assert all(k in t[0] for k in ("sym_teams=1", "bsym_wave=0", "cg_fold=7"))
        assert "sym_teams=2" in t[1] and "cg_fold=0" in t[1] and "bsym_wave=0" in t[1]
        for bad in ("default ld_pad=0", "n<=100 ld_pad=128", "default rows_bpc=99", "default nosuchkey=1",
                    "n<=0 rows_bpc=2", "default sym_teams=3", "default bsym_wave=2", "default cg_fold=8"):
            with pytest.raises(qpgpu.QpError):
                qpgpu.tune_set(bad)
    finally:
        qpgpu.tune_set(before)
    assert qpgpu.tune_get() == before


def test_committed_autotune_cache_parses():
    path = os.path.join(os.path.dirname(os.path.abspath(qpgpu.LIB_PATH)), "autotune_gfx950.txt")
    if not os.path.exists(path):
        pytest.skip("no autotune cache")
    before = qpgpu.tune_get()
    try:
        with open(path) as f:
            text = f.read()
        qpgpu.tune_set(text)  # accepted: layout keys equal to the built-in ones
        want = [ln.split()[0] for ln in text.splitlines() if ln.startswith("n<=")]
        assert [ln.split()[0] for ln in qpgpu.tune_get().splitlines()[1:]] == want
    finally:
        qpgpu.tune_set(before)


def test_hbm_read_probe_rejects_bad_arguments():
    ms = ct.c_double(0.0)
    L = qpgpu.lib()
    for nbytes, wg, reps in ((0, 8, 1), (17, 8, 1), (1 << 20, 0, 1), (1 << 20, 33, 1), (1 << 20, 8, 0)):
        assert L.qp_hbm_read_time(nbytes, wg, reps, ct.byref(ms)) == qpgpu.QP_E_INVALID
    assert L.qp_hbm_read_time(1 << 20, 8, 1, None) == qpgpu.QP_E_INVALID

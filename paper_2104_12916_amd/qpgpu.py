"""ctypes binding of libqpgpu.so (include/qpgpu.h), same names as the C ABI.

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Arrays are either NumPy float64 arrays (host memory, QP_MEM_HOST) or
torch float64 CUDA tensors (device memory, QP_MEM_DEVICE); the library is
loaded from the package directory and a missing build raises immediately.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqpgpu.so")

QP_OK, QP_E_INVALID, QP_E_NOT_SPD, QP_E_RANK, QP_E_NOCONV, QP_E_NOMEM, QP_E_DEVICE, QP_E_STATE = range(8)
QP_PREC_NONE, QP_PREC_LOW_DOF, QP_PREC_FEW_EQ, QP_PREC_AUTO = range(4)
QP_FP64, QP_MIXED = 0, 1
QP_MEM_HOST, QP_MEM_DEVICE = 0, 1
QP_KF_IMPLICIT, QP_KF_EXPLICIT = 0, 1
QP_PH_EXACT, QP_PH_DIAG = 0, 1

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "qp_default_options", "qp_setup", "qp_factor_K0", "qp_k0_solve", "qp_kf_apply",
    "qp_pcg_solve", "qp_ipm_solve", "qp_op_time", "qp_profile_get", "qp_ctx_bytes", "qp_destroy", "qp_status_str",
    "qp_last_error", "qp_batch_create", "qp_batch_admit", "qp_batch_step", "qp_batch_finished", "qp_batch_collect",
    "qp_batch_query", "qp_batch_footprint", "qp_batch_last_error", "qp_batch_destroy", "qp_batch_profile_get",
    "qp_k0_one_pass", "qp_c_identity", "qp_ipm_cg_steps",
    "qp_shared_setup", "qp_shared_pcg_solve", "qp_shared_ipm_solve", "qp_shared_last_error", "qp_shared_destroy",
    "qp_tune_set", "qp_tune_get", "qp_hbm_read_time", "qp_factor_K0_static", "qp_dense_time",
)
# bytes of the fixed device array qp_factor_K0_static takes its scratch from (QPGPU_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 64 << 20


class qp_options(ct.Structure):
    _fields_ = [
        ("rtol_kkt", ct.c_double), ("cg_theta", ct.c_double), ("cg_rtol", ct.c_double),
        ("tau", ct.c_double), ("max_ipm", ct.c_int), ("max_pcg", ct.c_int),
        ("poll_every", ct.c_int), ("prec", ct.c_int), ("precision", ct.c_int),
        ("verbose", ct.c_int), ("profile", ct.c_int), ("kf_form", ct.c_int), ("ph_form", ct.c_int),
        ("cg_graph", ct.c_int),
    ]


class qp_pcg_info(ct.Structure):
    _fields_ = [
        ("iters", ct.c_int), ("status", ct.c_int), ("rel_res", ct.c_double),
        ("refinements", ct.c_int), ("fp64_fallback", ct.c_int),
    ]


class qp_ipm_info(ct.Structure):
    _fields_ = [
        ("ipm_iters", ct.c_int), ("pcg_iters_total", ct.c_longlong), ("rel_kkt", ct.c_double),
        ("rel_kkt_parts", ct.c_double * 5), ("obj", ct.c_double), ("mu", ct.c_double),
        ("status", ct.c_int), ("refinements_total", ct.c_int), ("fp64_fallbacks", ct.c_int),
        ("t_solve_ms", ct.c_double), ("pcg_iters_fp64", ct.c_longlong),
    ]


_lib = None


def lib():
    """Load libqpgpu.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2104_12916_amd.build")
    L = ct.CDLL(LIB_PATH)
    P, I, D = ct.c_void_p, ct.c_int, ct.c_double
    L.qp_default_options.argtypes = [ct.POINTER(qp_options)]
    L.qp_default_options.restype = None
    L.qp_setup.argtypes = [ct.POINTER(P), I, I, I, P, P, P, P, P, P, I, ct.POINTER(qp_options), P]
    L.qp_factor_K0.argtypes = [P]
    L.qp_factor_K0_static.argtypes = [P]
    L.qp_k0_solve.argtypes = [P, P, P, I]
    L.qp_kf_apply.argtypes = [P, P, P, P, I]
    L.qp_pcg_solve.argtypes = [P, P, P, P, I, I, D, I, ct.POINTER(qp_pcg_info)]
    L.qp_ipm_solve.argtypes = [P, P, P, P, P, I, ct.POINTER(qp_ipm_info)]
    L.qp_op_time.argtypes = [P, I, I, I, ct.POINTER(D)]
    L.qp_profile_get.argtypes = [P, ct.POINTER(D), ct.POINTER(ct.c_longlong), I]
    L.qp_k0_one_pass.argtypes = [P]
    L.qp_k0_one_pass.restype = I
    L.qp_c_identity.argtypes = [P]
    L.qp_c_identity.restype = I
    L.qp_ipm_cg_steps.argtypes = [P, ct.POINTER(I), ct.POINTER(I), I, ct.POINTER(I)]
    L.qp_ipm_cg_steps.restype = I
    L.qp_ctx_bytes.argtypes = [P]
    L.qp_ctx_bytes.restype = ct.c_size_t
    L.qp_destroy.argtypes = [P]
    L.qp_destroy.restype = None
    L.qp_status_str.argtypes = [I]
    L.qp_status_str.restype = ct.c_char_p
    L.qp_last_error.argtypes = [P]
    L.qp_last_error.restype = ct.c_char_p
    LL, SZ = ct.c_longlong, ct.c_size_t
    L.qp_batch_create.argtypes = [ct.POINTER(P), ct.POINTER(qp_options), SZ, P]
    L.qp_batch_admit.argtypes = [P, I, I, I, P, P, P, P, P, P, I, ct.POINTER(LL)]
    L.qp_batch_step.argtypes = [P, I, ct.POINTER(I)]
    L.qp_batch_finished.argtypes = [P, ct.POINTER(LL), I, ct.POINTER(I)]
    L.qp_batch_collect.argtypes = [P, LL, P, P, P, P, I, ct.POINTER(qp_ipm_info)]
    L.qp_batch_query.argtypes = [P, ct.POINTER(I), ct.POINTER(I), ct.POINTER(SZ), ct.POINTER(SZ), ct.POINTER(LL)]
    L.qp_batch_footprint.argtypes = [ct.POINTER(qp_options), I, I, I]
    L.qp_batch_footprint.restype = SZ
    L.qp_batch_last_error.argtypes = [P]
    L.qp_batch_last_error.restype = ct.c_char_p
    L.qp_batch_profile_get.argtypes = [P, ct.POINTER(D), ct.POINTER(D), ct.POINTER(LL), I]
    L.qp_batch_destroy.argtypes = [P]
    L.qp_batch_destroy.restype = None
    L.qp_shared_setup.argtypes = [ct.POINTER(P), I, I, I, P, P, P, I, ct.POINTER(qp_options), P]
    L.qp_shared_pcg_solve.argtypes = [P, I, P, P, P, I, I, D, I, ct.POINTER(qp_pcg_info)]
    L.qp_shared_ipm_solve.argtypes = [P, I, P, P, P, P, P, P, P, I, ct.POINTER(qp_ipm_info)]
    L.qp_shared_last_error.argtypes = [P]
    L.qp_shared_last_error.restype = ct.c_char_p
    L.qp_shared_destroy.argtypes = [P]
    L.qp_shared_destroy.restype = None
    L.qp_tune_set.argtypes = [ct.c_char_p]
    L.qp_tune_get.argtypes = [ct.c_char_p, ct.c_size_t, ct.POINTER(ct.c_size_t)]
    L.qp_hbm_read_time.argtypes = [ct.c_size_t, I, I, ct.POINTER(D)]
    L.qp_dense_time.argtypes = [I, I, I, ct.POINTER(D)]
    for name in ("qp_setup", "qp_factor_K0", "qp_factor_K0_static", "qp_k0_solve", "qp_kf_apply", "qp_pcg_solve",
                 "qp_ipm_solve",
                 "qp_op_time", "qp_profile_get", "qp_batch_create", "qp_batch_admit", "qp_batch_step",
                 "qp_batch_finished", "qp_batch_collect", "qp_batch_query", "qp_batch_profile_get",
                 "qp_shared_setup", "qp_shared_pcg_solve", "qp_shared_ipm_solve", "qp_tune_set", "qp_tune_get",
                 "qp_hbm_read_time", "qp_dense_time"):
        getattr(L, name).restype = I
    _lib = L
    return L


# --- marshalling ------------------------------------------------------------
def _ptr(a):
    """(pointer, where) for a float64 NumPy array or torch CUDA tensor."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
            raise TypeError("host arrays must be C-contiguous float64")
        return a.ctypes.data_as(ct.c_void_p), QP_MEM_HOST
    try:
        import torch
    except ImportError as e:  # pragma: no cover
        raise TypeError("expected a numpy array") from e
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError("device tensors must be contiguous float64")
        if not a.is_cuda:
            raise TypeError("torch tensors must live on the GPU (use NumPy for host data)")
        return ct.c_void_p(a.data_ptr()), QP_MEM_DEVICE
    raise TypeError(f"unsupported array type {type(a)}")


def _has_tensor(*arrs) -> bool:
    return any(not isinstance(a, np.ndarray) for a in arrs)


def _torch_stream(*arrs):
    """torch's current stream (as an int) when any argument is a torch tensor and
    that stream is not the null stream, else None."""
    if not _has_tensor(*arrs):
        return None
    import torch
    return torch.cuda.current_stream().cuda_stream or None


def _wait_torch(*arrs) -> None:
    """Wait for torch's current stream when any argument is a torch tensor.

    The library reads device inputs (and writes device outputs) on its own stream,
    which waits for no other stream; this orders the call after the torch work that
    wrote the inputs or still reads the outputs."""
    if _has_tensor(*arrs):
        import torch
        torch.cuda.current_stream().synchronize()


def _where(*arrs):
    ws = {_ptr(a)[1] for a in arrs}
    if len(ws) != 1:
        raise TypeError("mix of host and device arrays in one call")
    return ws.pop()


def tune_get() -> str:
    """Current launch-shape table (the cache format of autotune.py)."""
    need = ct.c_size_t(0)
    lib().qp_tune_get(None, 0, ct.byref(need))
    buf = ct.create_string_buffer(need.value)
    st = lib().qp_tune_get(buf, need.value, ct.byref(need))
    if st != QP_OK:
        raise QpError(st, "qp_tune_get failed")
    return buf.value.decode()


def dense_time(op: int, n: int, reps: int = 10) -> float:
    """Average ms of one run of a factorization kernel of size n (qp_dense_time):
    op 0 GEMM n^3, op 1 GEMM with a triangular operand, op 2 Cholesky-inverse."""
    ms = ct.c_double(0.0)
    st = lib().qp_dense_time(op, n, reps, ct.byref(ms))
    if st != QP_OK:
        raise QpError(st, "qp_dense_time failed")
    return ms.value


def hbm_read_time(nbytes: int, wg_per_cu: int = 8, reps: int = 20) -> float:
    """Average ms of one streaming read of an nbytes device buffer (qp_hbm_read_time)."""
    ms = ct.c_double(0.0)
    st = lib().qp_hbm_read_time(nbytes, wg_per_cu, reps, ct.byref(ms))
    if st != QP_OK:
        raise QpError(st, "qp_hbm_read_time failed")
    return ms.value


def tune_set(spec: str) -> None:
    st = lib().qp_tune_set(spec.encode())
    if st != QP_OK:
        raise QpError(st, f"qp_tune_set rejected {spec!r}")


class QpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{qp_status_str(status)}: {msg}")
        self.status = status


def qp_default_options(**overrides) -> qp_options:
    o = qp_options()
    lib().qp_default_options(ct.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def qp_status_str(st: int) -> str:
    return lib().qp_status_str(int(st)).decode()


def qp_last_error(ctx) -> str:
    return lib().qp_last_error(ctx).decode()


def qp_setup(H, c, A, b, C, d, opt: qp_options | None = None, stream=None):
    """Returns (status, ctx).  stream: hipStream_t as int, or None (torch's current
    stream for torch tensors, else a stream owned by the context)."""
    n, m1, m2 = H.shape[0], A.shape[0], C.shape[0]
    where = _where(H, c, A, b, C, d)
    _wait_torch(H, c, A, b, C, d)
    if stream is None:
        stream = _torch_stream(H, c, A, b, C, d)
    ctx = ct.c_void_p()
    if opt is None:
        opt = qp_default_options()
    st = lib().qp_setup(ct.byref(ctx), n, m1, m2, *(_ptr(a)[0] for a in (H, c, A, b, C, d)), where,
                        ct.byref(opt), ct.c_void_p(stream) if stream else None)
    return st, ctx


def qp_factor_K0(ctx) -> int:
    return lib().qp_factor_K0(ctx)


def qp_factor_K0_static(ctx) -> int:
    return lib().qp_factor_K0_static(ctx)


def qp_k0_solve(ctx, rhs, out) -> int:
    _wait_torch(rhs, out)
    return lib().qp_k0_solve(ctx, _ptr(rhs)[0], _ptr(out)[0], _where(rhs, out))


def qp_kf_apply(ctx, dvec, p, q) -> int:
    _wait_torch(dvec, p, q)
    return lib().qp_kf_apply(ctx, _ptr(dvec)[0], _ptr(p)[0], _ptr(q)[0], _where(dvec, p, q))


def qp_pcg_solve(ctx, dvec, rhs, dnu, prec: int, rtol: float, maxit: int = 0):
    info = qp_pcg_info()
    _wait_torch(dvec, rhs, dnu)
    st = lib().qp_pcg_solve(ctx, _ptr(dvec)[0], _ptr(rhs)[0], _ptr(dnu)[0], _where(dvec, rhs, dnu), int(prec),
                            float(rtol), int(maxit), ct.byref(info))
    return st, info


def qp_ipm_solve(ctx, x, lam, nu, s):
    info = qp_ipm_info()
    _wait_torch(x, lam, nu, s)
    st = lib().qp_ipm_solve(ctx, _ptr(x)[0], _ptr(lam)[0], _ptr(nu)[0], _ptr(s)[0], _where(x, lam, nu, s),
                            ct.byref(info))
    return st, info


def qp_op_time(ctx, op: int, precision: int = QP_FP64, reps: int = 20):
    """Returns (status, average milliseconds per launch)."""
    ms = ct.c_double(0.0)
    st = lib().qp_op_time(ctx, int(op), int(precision), int(reps), ct.byref(ms))
    return st, ms.value


def qp_profile_get(ctx, reset: bool = False):
    """Returns (status, [avg ms per launch] * 6, [samples] * 6)."""
    ms = (ct.c_double * 6)()
    cnt = (ct.c_longlong * 6)()
    st = lib().qp_profile_get(ctx, ms, cnt, int(reset))
    return st, list(ms), list(cnt)


def qp_ctx_bytes(ctx) -> int:
    return int(lib().qp_ctx_bytes(ctx))


def qp_destroy(ctx) -> None:
    lib().qp_destroy(ctx)


# --- batches ------------------------------------------------------------------
def qp_batch_create(opt: qp_options | None = None, budget_bytes: int = 0, stream=None):
    """Returns (status, batch handle)."""
    b = ct.c_void_p()
    if opt is None:
        opt = qp_default_options()
    st = lib().qp_batch_create(ct.byref(b), ct.byref(opt), int(budget_bytes), ct.c_void_p(stream) if stream else None)
    return st, b


def qp_batch_admit(batch, H, c, A, b, C, d):
    """Returns (status, ticket).  Torch tensors: waits for torch's current stream
    first, since the batch reads them on its own stream."""
    n, m1, m2 = H.shape[0], A.shape[0], C.shape[0]
    where = _where(H, c, A, b, C, d)
    _wait_torch(H, c, A, b, C, d)
    t = ct.c_longlong(0)
    st = lib().qp_batch_admit(batch, n, m1, m2, *(_ptr(a)[0] for a in (H, c, A, b, C, d)), where, ct.byref(t))
    return st, t.value


def qp_batch_step(batch, max_rounds: int = 1):
    """Returns (status, finished-and-uncollected count)."""
    nd = ct.c_int(0)
    st = lib().qp_batch_step(batch, int(max_rounds), ct.byref(nd))
    return st, nd.value


def qp_batch_finished(batch, cap: int = 4096):
    """Returns (status, list of finished tickets)."""
    arr = (ct.c_longlong * max(cap, 1))()
    cnt = ct.c_int(0)
    st = lib().qp_batch_finished(batch, arr, int(cap), ct.byref(cnt))
    return st, [arr[k] for k in range(cnt.value)]


def qp_batch_collect(batch, ticket: int, x, lam, nu, s):
    """Returns (status of the QP, qp_ipm_info)."""
    info = qp_ipm_info()
    _wait_torch(x, lam, nu, s)
    st = lib().qp_batch_collect(batch, int(ticket), _ptr(x)[0], _ptr(lam)[0], _ptr(nu)[0], _ptr(s)[0],
                                _where(x, lam, nu, s), ct.byref(info))
    return st, info


def qp_batch_query(batch):
    """Returns (status, dict of the batch counters)."""
    a, f, r = ct.c_int(0), ct.c_int(0), ct.c_longlong(0)
    u, cap = ct.c_size_t(0), ct.c_size_t(0)
    st = lib().qp_batch_query(batch, ct.byref(a), ct.byref(f), ct.byref(u), ct.byref(cap), ct.byref(r))
    return st, {"in_flight": a.value, "finished": f.value, "bytes_used": u.value, "bytes_capacity": cap.value,
                "rounds": r.value}


def qp_batch_footprint(opt: qp_options | None, n: int, m1: int, m2: int) -> int:
    return int(lib().qp_batch_footprint(ct.byref(opt) if opt is not None else None, int(n), int(m1), int(m2)))


def qp_batch_last_error(batch) -> str:
    return lib().qp_batch_last_error(batch).decode()


def qp_batch_profile_get(batch, reset: bool = False):
    """Returns (status, [avg ms] * 6, [avg bytes] * 6, [samples] * 6)."""
    ms = (ct.c_double * 6)()
    by = (ct.c_double * 6)()
    cnt = (ct.c_longlong * 6)()
    st = lib().qp_batch_profile_get(batch, ms, by, cnt, int(reset))
    return st, list(ms), list(by), list(cnt)


def qp_batch_destroy(batch) -> None:
    lib().qp_batch_destroy(batch)


class Batch:
    """Owns one batch; admit/step/collect with NumPy host arrays."""

    def __init__(self, budget_bytes: int = 0, **opts):
        stream = opts.pop("stream", None)
        self.opt = qp_default_options(**opts)
        st, b = qp_batch_create(self.opt, budget_bytes, stream)
        if st != QP_OK:
            raise QpError(st, "qp_batch_create failed")
        self.b = b
        self.sizes = {}

    def admit(self, H, c, A, b, C, d):
        """Ticket, or None when the batch has no room now (QP_E_NOMEM)."""
        st, t = qp_batch_admit(self.b, H, c, A, b, C, d)
        if st == QP_E_NOMEM:
            return None
        if st != QP_OK:
            raise QpError(st, qp_batch_last_error(self.b))
        self.sizes[t] = (H.shape[0], A.shape[0], C.shape[0])
        return t

    def footprint(self, n: int, m1: int, m2: int) -> int:
        """Arena bytes a QP of these sizes takes under this batch's options."""
        return qp_batch_footprint(self.opt, n, m1, m2)

    def step(self, rounds: int = 1) -> int:
        st, nd = qp_batch_step(self.b, rounds)
        if st != QP_OK:
            raise QpError(st, qp_batch_last_error(self.b))
        return nd

    def finished(self):
        st, t = qp_batch_finished(self.b)
        if st != QP_OK:
            raise QpError(st, qp_batch_last_error(self.b))
        return t

    def collect(self, ticket, accept=(QP_OK,)):
        n, m1, m2 = self.sizes.pop(ticket)
        x, lam, nu, s = np.zeros(n), np.zeros(m1), np.zeros(m2), np.zeros(m2)
        st, info = qp_batch_collect(self.b, ticket, x, lam, nu, s)
        if st not in accept:
            raise QpError(st, qp_batch_last_error(self.b))
        return x, lam, nu, s, info

    def query(self):
        return qp_batch_query(self.b)[1]

    def profile(self, reset=False):
        st, ms, by, cnt = qp_batch_profile_get(self.b, reset)
        if st != QP_OK:
            raise QpError(st, qp_batch_last_error(self.b))
        return ms, by, cnt

    def close(self):
        if self.b:
            qp_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Shared:
    """QPs sharing H, A and C (qp_shared_*): one K0 factorization, block PCG over k QPs."""

    def __init__(self, H, A, C, **opts):
        stream = opts.pop("stream", None)
        self.opt = qp_default_options(**opts)
        self.n, self.m1, self.m2 = H.shape[0], A.shape[0], C.shape[0]
        (ph, where), (pa, _), (pc, _) = _ptr(H), _ptr(A), _ptr(C)
        _where(H, A, C)
        _wait_torch(H, A, C)
        if stream is None:
            stream = _torch_stream(H, A, C)
        out = ct.c_void_p()
        st = lib().qp_shared_setup(ct.byref(out), self.n, self.m1, self.m2, ph, pa, pc, where, ct.byref(self.opt),
                                   stream)
        if st != QP_OK:
            raise QpError(st, "qp_shared_setup failed")
        self.sh = out

    def check(self, st, accept=(QP_OK,)):
        if st not in accept:
            raise QpError(st, (lib().qp_shared_last_error(self.sh) or b"").decode())

    def pcg(self, dvecs, rhss, prec=QP_PREC_LOW_DOF, rtol=1e-10, maxit=0, accept=(QP_OK,)):
        """dvecs, rhss: k x m2.  Returns (dnu k x m2, [qp_pcg_info] * k)."""
        dv = np.ascontiguousarray(dvecs, dtype=np.float64)
        rh = np.ascontiguousarray(rhss, dtype=np.float64)
        k = dv.shape[0]
        out = np.zeros_like(rh)
        infos = (qp_pcg_info * k)()
        st = lib().qp_shared_pcg_solve(self.sh, k, _ptr(dv)[0], _ptr(rh)[0], _ptr(out)[0], QP_MEM_HOST, int(prec),
                                       float(rtol), int(maxit), infos)
        self.check(st, accept)
        return out, list(infos)

    def ipm(self, cs, bs, ds, accept=(QP_OK,)):
        """cs: k x n, bs: k x m1, ds: k x m2.  Returns (x, lam, nu, s, [qp_ipm_info] * k)."""
        c = np.ascontiguousarray(cs, dtype=np.float64)
        b = np.ascontiguousarray(bs, dtype=np.float64)
        d = np.ascontiguousarray(ds, dtype=np.float64)
        k = c.shape[0]
        x, lam = np.zeros((k, self.n)), np.zeros((k, self.m1))
        nu, s = np.zeros((k, self.m2)), np.zeros((k, self.m2))
        infos = (qp_ipm_info * k)()
        st = lib().qp_shared_ipm_solve(self.sh, k, _ptr(c)[0], _ptr(b)[0], _ptr(d)[0], _ptr(x)[0], _ptr(lam)[0],
                                       _ptr(nu)[0], _ptr(s)[0], QP_MEM_HOST, infos)
        self.check(st, accept)
        return x, lam, nu, s, list(infos)

    def close(self):
        if getattr(self, "sh", None):
            lib().qp_shared_destroy(self.sh)
            self.sh = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- convenience wrapper used by tests and the benchmark --------------------
class Solver:
    """Owns one context; raises QpError on any non-OK status it is not told to accept."""

    def __init__(self, H, c, A, b, C, d, **opts):
        self.n, self.m1, self.m2 = H.shape[0], A.shape[0], C.shape[0]
        stream = opts.pop("stream", None)
        self.opt = qp_default_options(**opts)
        st, ctx = qp_setup(H, c, A, b, C, d, self.opt, stream)
        if st != QP_OK:
            raise QpError(st, "qp_setup failed")
        self.ctx = ctx

    def check(self, st, accept=(QP_OK,)):
        if st not in accept:
            raise QpError(st, qp_last_error(self.ctx))
        return st

    def factor(self, static=False):
        """qp_factor_K0, or with static=True qp_factor_K0_static (no device allocation)."""
        return self.check((qp_factor_K0_static if static else qp_factor_K0)(self.ctx))

    def k0_solve(self, rhs):
        out = np.empty_like(rhs)
        self.check(qp_k0_solve(self.ctx, rhs, out))
        return out

    def kf_apply(self, dvec, p):
        q = np.empty_like(p)
        self.check(qp_kf_apply(self.ctx, dvec, p, q))
        return q

    def pcg(self, dvec, rhs, prec=QP_PREC_LOW_DOF, rtol=1e-10, maxit=0, accept=(QP_OK,)):
        dnu = np.empty_like(rhs)
        st, info = qp_pcg_solve(self.ctx, dvec, rhs, dnu, prec, rtol, maxit)
        self.check(st, accept)
        return dnu, info

    def ipm(self, accept=(QP_OK,)):
        x = np.empty(self.n)
        lam = np.empty(self.m1)
        nu = np.empty(self.m2)
        s = np.empty(self.m2)
        st, info = qp_ipm_solve(self.ctx, x, lam, nu, s)
        self.check(st, accept)
        return x, lam, nu, s, info

    def op_time(self, op, precision=QP_FP64, reps=20):
        st, ms = qp_op_time(self.ctx, op, precision, reps)
        self.check(st)
        return ms

    def profile(self, reset=False):
        st, ms, cnt = qp_profile_get(self.ctx, reset)
        self.check(st)
        return ms, cnt

    def k0_one_pass(self):
        """True if the CG step forms M^T Sigma M u in one pass over M."""
        return bool(lib().qp_k0_one_pass(self.ctx))

    def cg_steps(self):
        """(predictor, corrector) CG steps of every IPM iteration of the last ipm()."""
        cnt = ct.c_int(0)
        st = lib().qp_ipm_cg_steps(self.ctx, None, None, 0, ct.byref(cnt))
        self.check(st)
        k = cnt.value
        a, b = (ct.c_int * max(k, 1))(), (ct.c_int * max(k, 1))()
        self.check(lib().qp_ipm_cg_steps(self.ctx, a, b, k, ct.byref(cnt)))
        return list(a[:k]), list(b[:k])

    def c_identity(self):
        """True once qp_factor_K0 has found C = I (the CG step then has no product by C)."""
        return bool(lib().qp_c_identity(self.ctx))

    def bytes(self):
        return qp_ctx_bytes(self.ctx)

    def close(self):
        if self.ctx:
            qp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

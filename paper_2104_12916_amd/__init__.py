"""MI355X (gfx950) implementation of the preconditioned implicit-PCG interior point
method of Karim & Solomonik (arXiv 2104.12916).

The solver lives in the HIP library ``libqpgpu.so`` (C ABI in include/qpgpu.h);
``paper_2104_12916_amd.qpgpu`` is its ctypes binding with the same names.
"""
from .qpgpu import (  # noqa: F401
    Solver, QpError, lib, qp_default_options, qp_setup, qp_factor_K0, qp_k0_solve, qp_kf_apply,
    qp_pcg_solve, qp_ipm_solve, qp_op_time, qp_profile_get, qp_ctx_bytes, qp_destroy, qp_status_str, qp_last_error,
    QP_OK, QP_E_INVALID, QP_E_NOT_SPD, QP_E_RANK, QP_E_NOCONV, QP_E_NOMEM, QP_E_DEVICE, QP_E_STATE,
    QP_PREC_NONE, QP_PREC_LOW_DOF, QP_PREC_FEW_EQ, QP_PREC_AUTO, QP_FP64, QP_MIXED,
    QP_MEM_HOST, QP_MEM_DEVICE, EXPORTS,
)

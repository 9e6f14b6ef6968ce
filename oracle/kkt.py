"""KKT residuals and the relative KKT score (oracle; test infrastructure only).

Follows the Lagrangian of eq. lagrangian and the optimality conditions of Sec. 2:
    H x + c - A^T lam - C^T nu = 0,  A x = b,  C x >= d,  nu >= 0,
    nu^T (C x - d) = 0.
"""
from __future__ import annotations

import numpy as np


def objective(qp, x) -> float:
    """f(x) = 1/2 x^T H x + c^T x (eq. qp)."""
    return float(0.5 * x @ (qp.H @ x) + qp.c @ x)


def dual_objective(qp, x, lam, nu) -> float:
    """Lagrangian dual value at a stationary point: -1/2 x^T H x + b^T lam + d^T nu.

    Substituting H x + c = A^T lam + C^T nu into the Lagrangian of eq. lagrangian
    gives this expression; weak duality makes primal minus dual equal
    lam^T (A x - b) + nu^T (C x - d) when stationarity holds.
    """
    return float(-0.5 * x @ (qp.H @ x) + qp.b @ lam + qp.d @ nu)


def rel_kkt(qp, x, lam, nu):
    """Slack-free relative KKT score of a candidate (x, lam, nu).

    Returns (score, parts) where score = max(parts.values()) and
      rho_d   : ||H x + c - A^T lam - C^T nu||_inf / (1 + max of the term norms)
      rho_e   : ||A x - b||_inf / (1 + max(||A x||_inf, ||b||_inf))
      rho_p   : ||max(d - C x, 0)||_inf / (1 + ||d||_inf)
      rho_gap : |f(x) - dual| / (1 + |f(x)|)
      rho_nu  : max(-nu) / (1 + ||nu||_inf), clipped at 0 (dual feasibility nu >= 0)
    """
    x = np.asarray(x, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    Hx = qp.H @ x
    ATl = qp.A.T @ lam
    CTn = qp.C.T @ nu
    rd = Hx + qp.c - ATl - CTn
    Ax = qp.A @ x
    Cx = qp.C @ x
    inf = lambda v: float(np.max(np.abs(v))) if v.size else 0.0  # noqa: E731
    rho_d = inf(rd) / (1.0 + max(inf(Hx), inf(qp.c), inf(ATl), inf(CTn)))
    rho_e = inf(Ax - qp.b) / (1.0 + max(inf(Ax), inf(qp.b)))
    rho_p = (float(np.max(np.maximum(qp.d - Cx, 0.0))) if Cx.size else 0.0) / (1.0 + inf(qp.d))
    pobj = objective(qp, x)
    dobj = dual_objective(qp, x, lam, nu)
    rho_gap = abs(pobj - dobj) / (1.0 + abs(pobj))
    rho_nu = max(0.0, float(np.max(-nu)) if nu.size else 0.0) / (1.0 + inf(nu))
    parts = dict(rho_d=rho_d, rho_e=rho_e, rho_p=rho_p, rho_gap=rho_gap, rho_nu=rho_nu)
    return max(parts.values()), parts


def newton_residuals(qp, x, lam, nu, s):
    """Residuals of eq. rhs-KKT4 without the centering term.

    r_g = -H x - c + A^T lam + C^T nu,  r_e = A x - b,  r_i = C x - d - s.
    """
    r_g = -(qp.H @ x) - qp.c + qp.A.T @ lam + qp.C.T @ nu
    r_e = qp.A @ x - qp.b
    r_i = qp.C @ x - qp.d - s
    return r_g, r_e, r_i

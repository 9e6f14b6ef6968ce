"""Full-system primal-dual interior point method (oracle; test infrastructure only).

The result is the unique minimizer of the strictly convex QP of eq. qp (H SPD,
A of full row rank, Sec. 1) together with its multipliers.  Each Newton step
solves the unreduced block system of eq. nonsym-indef-KKT

    [ H  -A^T  -C^T   0 ] [dx  ]     [ H x + c - A^T lam - C^T nu ]
    [ A    0     0    0 ] [dlam] = - [ A x - b                    ]
    [ C    0     0   -I ] [dnu ]     [ C x - d - s                ]
    [ 0    0     S    V ] [ds  ]     [ S V e - sigma mu e         ]

by one dense LU factorization per iteration, so it never uses the reduced
system that the GPU path solves.

The paper fixes the central-path system (eqs. nonlinear, duality) and leaves the
centering and step rules open.  This oracle takes Mehrotra's predictor-corrector
reading:
  * initial point: (x0, lam0) solves the equality-only QP
        [H -A^T; A 0] [x; lam] = [-c; b];   s0 = max(C x0 - d, 1);  nu0 = 1;
  * predictor: sigma = 0; alpha_aff = largest alpha <= 1 keeping s, nu >= 0;
    mu_aff = (s + a ds)^T (nu + a dnu) / m2;  sigma = (mu_aff / mu)^3;
  * corrector: last block of the right-hand side becomes
        S V e + dS_aff dV_aff e - sigma mu e;
  * step: alpha = min(1, tau alpha_max), tau = 0.995, one alpha for primal and
    dual;  stop when the relative KKT score (oracle.kkt.rel_kkt) <= tol.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .kkt import rel_kkt, objective, newton_residuals


class OracleInputError(ValueError):
    pass


@dataclass
class IPMResult:
    x: np.ndarray
    lam: np.ndarray
    nu: np.ndarray
    s: np.ndarray
    obj: float
    iters: int
    rel_kkt: float
    parts: dict
    converged: bool
    history: list = field(default_factory=list)


def validate(qp, sym_tol: float = 1e-14):
    """Assumptions of Sec. 1: H symmetric positive definite, 0 < m1 <= n, rank A = m1."""
    H, A = qp.H, qp.A
    n, m1 = H.shape[0], A.shape[0]
    if not (0 < m1 <= n):
        raise OracleInputError("need 0 < m1 <= n")
    if np.linalg.norm(H - H.T) > sym_tol * max(1.0, np.linalg.norm(H)):
        raise OracleInputError("H is not symmetric")
    try:
        np.linalg.cholesky(H)
    except np.linalg.LinAlgError as e:
        raise OracleInputError("H is not positive definite") from e
    sv = np.linalg.svd(A, compute_uv=False)
    if sv[-1] <= max(A.shape) * np.finfo(float).eps * sv[0]:
        raise OracleInputError("A is rank deficient")


def initial_point(qp):
    """Equality-only QP solution, then s0 = max(C x0 - d, 1) and nu0 = 1."""
    n, m1 = qp.n, qp.m1
    K = np.zeros((n + m1, n + m1))
    K[:n, :n] = qp.H
    K[:n, n:] = -qp.A.T
    K[n:, :n] = qp.A
    sol = sla.solve(K, np.concatenate([-qp.c, qp.b]))
    x, lam = sol[:n], sol[n:]
    s = np.maximum(qp.C @ x - qp.d, 1.0)
    nu = np.ones(qp.m2)
    return x, lam, nu, s


def max_step(v, dv) -> float:
    """Largest alpha >= 0 with v + alpha dv >= 0 (inf when dv >= 0)."""
    neg = dv < 0
    if not np.any(neg):
        return np.inf
    return float(np.min(-v[neg] / dv[neg]))


def centering(mu, mu_aff) -> float:
    """Mehrotra's centering parameter sigma = (mu_aff / mu)^3 (sigma of eq. nonlinear)."""
    return (mu_aff / mu) ** 3


def corrector_rc(s, nu, ds_aff, dnu_aff, sigma, mu):
    """Last block of the corrector right-hand side: S V e + dS_aff dV_aff e - sigma mu e.

    The complementarity row of eq. nonsym-indef-KKT with Mehrotra's second-order term.
    """
    return s * nu + ds_aff * dnu_aff - sigma * mu


def newton_matrix(qp, nu, s):
    """Coefficient matrix of eq. nonsym-indef-KKT at (nu, s)."""
    n, m1, m2 = qp.n, qp.m1, qp.m2
    N = n + m1 + 2 * m2
    K = np.zeros((N, N))
    i1, i2, i3 = n, n + m1, n + m1 + m2
    K[:i1, :i1] = qp.H
    K[:i1, i1:i2] = -qp.A.T
    K[:i1, i2:i3] = -qp.C.T
    K[i1:i2, :i1] = qp.A
    K[i2:i3, :i1] = qp.C
    K[i2:i3, i3:] = -np.eye(m2)
    K[i3:, i2:i3] = np.diag(s)
    K[i3:, i3:] = np.diag(nu)
    return K


def solve(qp, tol: float = 1e-10, max_iter: int = 200, tau: float = 0.995,
          check: bool = True, max_iters_cap: int | None = None) -> IPMResult:
    """Run the full-system IPM to rel_kkt <= tol (or max_iter iterations).

    ``max_iters_cap`` stops after that many iterations regardless of
    convergence (used to time a bounded sample).
    """
    if check:
        validate(qp)
    n, m1, m2 = qp.n, qp.m1, qp.m2
    x, lam, nu, s = initial_point(qp)
    hist = []
    sc, parts = rel_kkt(qp, x, lam, nu)
    it = 0
    converged = sc <= tol
    limit = max_iter if max_iters_cap is None else min(max_iter, max_iters_cap)
    while not converged and it < limit:
        # residuals of eq. rhs-KKT4; the first row of eq. nonsym-indef-KKT carries -r_g
        r_g, r_e, r_i = newton_residuals(qp, x, lam, nu, s)
        mu = float(s @ nu) / m2
        lu = sla.lu_factor(newton_matrix(qp, nu, s))
        base = np.concatenate([-r_g, r_e, r_i])

        def split(sol):
            return (sol[:n], sol[n:n + m1], sol[n + m1:n + m1 + m2], sol[n + m1 + m2:])

        # predictor (affine scaling, sigma = 0)
        aff = split(sla.lu_solve(lu, -np.concatenate([base, s * nu])))
        dx_a, dl_a, dn_a, ds_a = aff
        a_aff = min(1.0, max_step(s, ds_a), max_step(nu, dn_a))
        mu_aff = float((s + a_aff * ds_a) @ (nu + a_aff * dn_a)) / m2
        sigma = centering(mu, mu_aff)
        # corrector
        rc = corrector_rc(s, nu, ds_a, dn_a, sigma, mu)
        dx, dl, dn, ds = split(sla.lu_solve(lu, -np.concatenate([base, rc])))
        a_max = min(max_step(s, ds), max_step(nu, dn))
        alpha = min(1.0, tau * a_max)
        x = x + alpha * dx
        lam = lam + alpha * dl
        nu = nu + alpha * dn
        s = s + alpha * ds
        it += 1
        sc, parts = rel_kkt(qp, x, lam, nu)
        hist.append(dict(it=it, mu=mu, sigma=sigma, alpha=alpha, rel_kkt=sc))
        converged = sc <= tol
        if not np.all(np.isfinite(x)) or alpha < 1e-14:
            break
    return IPMResult(x, lam, nu, s, objective(qp, x), it, sc, parts, bool(converged), hist)

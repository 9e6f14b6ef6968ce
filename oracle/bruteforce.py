"""Active-set enumeration for tiny QPs (oracle pin; test infrastructure only).

For a strictly convex QP (eq. qp with H SPD) the minimizer is the unique point
satisfying the KKT conditions of Sec. 2.  Guessing the active inequality set W
turns those conditions into one linear system

    [ H   -A^T  -C_W^T ] [x   ]   [ -c  ]
    [ A    0     0     ] [lam ] = [  b  ]
    [ C_W  0     0     ] [nu_W]   [ d_W ]

whose solution is optimal iff C x >= d and nu_W >= 0.  Trying every W with
|W| <= n - m1 (more active rows than degrees of freedom would be dependent)
finds it without any interior point machinery.
"""
from __future__ import annotations

import itertools

import numpy as np


def solve(qp, feas_tol: float = 1e-12, dual_tol: float = 1e-12):
    """Return (x, lam, nu, W) of the KKT point found by enumeration."""
    n, m1, m2 = qp.n, qp.m1, qp.m2
    best = None
    for k in range(0, min(m2, n - m1) + 1):
        for W in itertools.combinations(range(m2), k):
            W = list(W)
            CW = qp.C[W, :]
            N = n + m1 + k
            K = np.zeros((N, N))
            K[:n, :n] = qp.H
            K[:n, n:n + m1] = -qp.A.T
            K[:n, n + m1:] = -CW.T
            K[n:n + m1, :n] = qp.A
            K[n + m1:, :n] = CW
            if np.linalg.matrix_rank(K) < N:
                continue
            sol = np.linalg.solve(K, np.concatenate([-qp.c, qp.b, qp.d[W]]))
            x, lam, nuW = sol[:n], sol[n:n + m1], sol[n + m1:]
            slack = qp.C @ x - qp.d
            scale = 1.0 + np.max(np.abs(qp.d))
            if np.min(slack, initial=np.inf) < -feas_tol * scale:
                continue
            if nuW.size and np.min(nuW) < -dual_tol * (1.0 + np.max(np.abs(nuW))):
                continue
            nu = np.zeros(m2)
            nu[W] = nuW
            f = 0.5 * x @ qp.H @ x + qp.c @ x
            if best is None or f < best[0] - 1e-14:
                best = (f, x, lam, nu, W)
    if best is None:
        raise RuntimeError("no KKT point found (infeasible QP?)")
    _, x, lam, nu, W = best
    return x, lam, nu, W

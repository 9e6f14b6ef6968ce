"""The inequality-constraint reduced system on explicit matrices (oracle only).

Everything here is a plain definition from Sec. 4 of the paper, written with
dense float64 NumPy/SciPy solves.  It is what the GPU path computes implicitly,
spelled out so that tests can compare the two element by element.

Sign convention.  The paper's fixed block is F = [-H A^T; A 0] (eq. f-def).  The
GPU path factorizes K0 = [H A^T; A 0] = -J F J with J = diag(-I_n, I_m1), so that
[C 0] F^{-1} [C^T; 0] = -[C 0] K0^{-1} [C^T; 0]; both forms are provided and a
test checks that they agree.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# --- fixed blocks ---------------------------------------------------------
def F_matrix(qp):
    """F = [-H A^T; A 0] (eq. f-def)."""
    n, m1 = qp.n, qp.m1
    F = np.zeros((n + m1, n + m1))
    F[:n, :n] = -qp.H
    F[:n, n:] = qp.A.T
    F[n:, :n] = qp.A
    return F


def K0_matrix(qp):
    """K0 = [H A^T; A 0] = -J F J."""
    n, m1 = qp.n, qp.m1
    K = np.zeros((n + m1, n + m1))
    K[:n, :n] = qp.H
    K[:n, n:] = qp.A.T
    K[n:, :n] = qp.A
    return K


def _C0(qp):
    """[C 0] (m2 x (n + m1))."""
    return np.hstack([qp.C, np.zeros((qp.m2, qp.m1))])


# --- the reduced matrix ---------------------------------------------------
def kf_explicit(qp, dvec):
    """K_F = D - [C 0] F^{-1} [C^T; 0] (eq. ineq-const-reduced)."""
    C0 = _C0(qp)
    X = sla.solve(F_matrix(qp), C0.T)
    K = np.diag(dvec) - C0 @ X
    return 0.5 * (K + K.T)


def kf_from_k0(qp, dvec):
    """K_F = D + [C 0] K0^{-1} [C^T; 0] (the same matrix through K0 = -J F J)."""
    C0 = _C0(qp)
    X = sla.solve(K0_matrix(qp), C0.T)
    K = np.diag(dvec) + C0 @ X
    return 0.5 * (K + K.T)


def kf_schur_form(qp, dvec):
    """K_F = D + C H^{-1} (H - Hbar_A) H^{-1} C^T, Hbar_A = A^T (A H^{-1} A^T)^{-1} A.

    The block-inverse expression of eqs. f-inv and schur-R.
    """
    Hinv = np.linalg.inv(qp.H)
    FH = qp.A @ Hinv @ qp.A.T
    HbarA = qp.A.T @ np.linalg.solve(FH, qp.A)
    K = np.diag(dvec) + qp.C @ Hinv @ (qp.H - HbarA) @ Hinv @ qp.C.T
    return 0.5 * (K + K.T)


def hbar_a(qp):
    """Hbar_A = A^T (A H^{-1} A^T)^{-1} A (Lemma lem_s_a)."""
    Hinv = np.linalg.inv(qp.H)
    return qp.A.T @ np.linalg.solve(qp.A @ Hinv @ qp.A.T, qp.A)


def k0_solve(qp, rhs):
    """K0^{-1} rhs by dense LU."""
    return sla.solve(K0_matrix(qp), rhs)


def kf_apply(qp, dvec, p):
    """K_F p = D p + [C 0] K0^{-1} [C^T p; 0] without forming K_F."""
    u = np.concatenate([qp.C.T @ p, np.zeros(qp.m1)])
    y = k0_solve(qp, u)[:qp.n]
    return dvec * p + qp.C @ y


# --- preconditioners ------------------------------------------------------
def P_L(dvec):
    """Low-degree-of-freedom preconditioner P_L = D (eq. preconditioner-1)."""
    return np.diag(dvec)


def ph_T(qp):
    """T = C H^{-1} C^T, the fixed part of P_H."""
    return qp.C @ sla.cho_solve(sla.cho_factor(qp.H, lower=True), qp.C.T)


def P_H(qp, dvec):
    """High-degree-of-freedom preconditioner P_H = D + C H^{-1} C^T (eq. preconditioner-2)."""
    T = ph_T(qp)
    return np.diag(dvec) + 0.5 * (T + T.T)


def ph_T_diag(qp):
    """T = C diag(H)^{-1} C^T: the P_H of the PH-KF cost model and experiments (Sec. 5.2)."""
    return (qp.C / np.diag(qp.H)) @ qp.C.T


def P_H_diag(qp, dvec):
    """P_H with H replaced by its diagonal: D + C diag(H)^{-1} C^T (Sec. 5.2)."""
    T = ph_T_diag(qp)
    return np.diag(dvec) + 0.5 * (T + T.T)


def preconditioned_eigs(K, P):
    """Eigenvalues of P^{-1/2} K P^{-1/2} (split preconditioning, Sec. 4.3)."""
    w, V = np.linalg.eigh(P)
    Pmh = (V / np.sqrt(w)) @ V.T
    M = Pmh @ K @ Pmh
    return np.linalg.eigvalsh(0.5 * (M + M.T))


# --- IPM pieces of the reduced formulation --------------------------------
def reduced_rhs(qp, x, lam, nu, s, rc):
    """r_nu = -r_a + [C 0] F^{-1} [r_g; r_e] (eq. ineq-const-reduced).

    r_g, r_e, r_i from eq. rhs-KKT4; rc is the complementarity residual
    (S V e - sigma mu e, or its corrector form); r_a = r_i + V^{-1} r_c (eq. augmented).
    """
    r_g = -(qp.H @ x) - qp.c + qp.A.T @ lam + qp.C.T @ nu
    r_e = qp.A @ x - qp.b
    r_i = qp.C @ x - qp.d - s
    r_a = r_i + rc / nu
    sol = sla.solve(F_matrix(qp), np.concatenate([r_g, r_e]))
    return -r_a + qp.C @ sol[:qp.n], (r_g, r_e, r_i, r_a)


def recover(qp, nu, rc, r_g, r_e, dnu):
    """(dx, dlam) from F [dx; dlam] = -[r_g + C^T dnu; r_e] (eq. schur-delta-x);
    ds = -V^{-1} r_c - D dnu (eq. delz) with D = V^{-1} S."""
    n = qp.n
    sol = sla.solve(F_matrix(qp), -np.concatenate([r_g + qp.C.T @ dnu, r_e]))
    return sol[:n], sol[n:]


def reduced_newton_step(qp, x, lam, nu, s, rc):
    """Newton direction through the reduced system solved directly (Cholesky).

    Returns (dx, dlam, dnu, ds).  Equal, in exact arithmetic, to the solution of
    eq. nonsym-indef-KKT with the same complementarity residual rc.
    """
    dvec = s / nu
    rnu, (r_g, r_e, r_i, r_a) = reduced_rhs(qp, x, lam, nu, s, rc)
    K = kf_explicit(qp, dvec)
    dnu = sla.cho_solve(sla.cho_factor(K, lower=True), rnu)
    dx, dlam = recover(qp, nu, rc, r_g, r_e, dnu)
    ds = -rc / nu - dvec * dnu
    return dx, dlam, dnu, ds


# --- textbook PCG (Sec. 6 protocol: zero initial guess, relative residual) -
def pcg(apply_K, rhs, apply_Pinv, tol: float, maxit: int):
    """Left-preconditioned conjugate gradient from a zero initial guess.

    Stops when ||r||_2 <= tol ||rhs||_2 (recursive residual).  Returns
    (x, iterations, residual norms).
    """
    x = np.zeros_like(rhs)
    r = rhs.copy()
    bnorm = float(np.linalg.norm(rhs))
    hist = [float(np.linalg.norm(r))]
    if bnorm == 0.0:
        return x, 0, hist
    z = apply_Pinv(r)
    p = z.copy()
    rho = float(r @ z)
    k = 0
    while k < maxit and hist[-1] > tol * bnorm:
        q = apply_K(p)
        alpha = rho / float(p @ q)
        x += alpha * p
        r -= alpha * q
        k += 1
        hist.append(float(np.linalg.norm(r)))
        if hist[-1] <= tol * bnorm:
            break
        z = apply_Pinv(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, k, hist

"""Pins of the CPU oracle against facts other than itself (no GPU).

Each test ties one oracle function to the mathematics or to the paper:
brute-force active sets, a closed-form box QP, exact reformulation identities
(Sec. 4.1), the rank lemmas and spectral theorems (Sec. 4.3), the CG iteration
corollaries, the inertia of F and generator determinism.  The mutation tests at
the end plant plausible mistakes in the oracle and check that a pin catches them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import boxqp, bruteforce, ipm, kkt, reduced


# --- P9 generator ------------------------------------------------------------
def test_generator_is_deterministic_and_feasible():
    a = synth.gaussian_qp(7, 40, 10, 25)
    b = synth.gaussian_qp(7, 40, 10, 25)
    for u, v in zip(a.arrays(), b.arrays()):
        assert np.array_equal(u, v)
    slack = a.C @ a.x0 - a.d
    assert np.all(slack >= 0.1 - 1e-12) and np.all(slack <= 1.0 + 1e-12)
    assert np.allclose(a.A @ a.x0, a.b, rtol=0, atol=1e-12)
    assert np.array_equal(a.H, a.H.T)
    assert np.all(np.linalg.eigvalsh(a.H) >= 1e-2 - 1e-10)


def test_illcond_generator_spectrum():
    q = synth.illcond_qp(3, 64, 8, 64)
    w = np.linalg.eigvalsh(q.H)
    assert np.allclose(w, np.logspace(-4, 2, 64), rtol=1e-8)


# --- P1 brute force ------------------------------------------------------------
@pytest.mark.parametrize("seed,n,m1,m2", [(0, 5, 2, 8), (1, 4, 1, 6), (2, 6, 3, 10), (3, 3, 1, 5),
                                          (4, 6, 2, 9), (5, 2, 1, 4)])
def test_ipm_matches_active_set_enumeration(seed, n, m1, m2):
    qp = synth.tiny_qp(seed, n, m1, m2)
    xb, lb, nb, W = bruteforce.solve(qp)
    r = ipm.solve(qp, tol=1e-12)
    assert r.converged
    assert np.max(np.abs(r.x - xb)) <= 1e-8 * (1 + np.max(np.abs(xb)))
    fb = kkt.objective(qp, xb)
    assert abs(r.obj - fb) <= 1e-10 * max(1.0, abs(fb))


# --- P2 closed form ------------------------------------------------------------
@pytest.mark.parametrize("seed,n,m1", [(0, 10, 3), (1, 16, 5), (2, 7, 1)])
def test_ipm_matches_closed_form_box_qp(seed, n, m1):
    qp = synth.box_qp(seed, n, m1)
    xc, lc, nc = boxqp.solve(qp)
    # the closed form itself satisfies every KKT condition exactly
    sc, parts = kkt.rel_kkt(qp, xc, lc, nc)
    assert sc <= 1e-14
    r = ipm.solve(qp, tol=1e-12)
    assert r.converged
    assert np.max(np.abs(r.x - xc)) <= 1e-8
    assert np.max(np.abs(r.lam - lc)) <= 1e-8
    assert np.max(np.abs(r.nu - nc)) <= 1e-8
    # the box QP activates both bound types (so the pin exercises nu_l and nu_u)
    nf = n - m1
    assert np.any(nc[:nf] > 1e-6) and np.any(nc[nf:] > 1e-6)


def test_rel_kkt_detects_each_violation():
    qp = synth.box_qp(1, 16, 5)
    x, lam, nu = boxqp.solve(qp)
    base, _ = kkt.rel_kkt(qp, x, lam, nu)
    assert base <= 1e-14
    e = 1e-3
    _, p = kkt.rel_kkt(qp, x + e, lam, nu)          # primal move: dual + equality residuals
    assert p["rho_d"] > 1e-5 and p["rho_e"] > 1e-5
    _, p = kkt.rel_kkt(qp, x, lam + e, nu)          # equality multiplier: dual residual
    assert p["rho_d"] > 1e-5
    nu2 = nu.copy()
    nu2[np.argmax(nu)] += e
    _, p = kkt.rel_kkt(qp, x, lam, nu2)             # dual residual and gap
    assert p["rho_d"] > 1e-6 and p["rho_gap"] > 1e-7
    nu3 = nu.copy()
    nu3[np.argmin(nu)] = -e
    _, p = kkt.rel_kkt(qp, x, lam, nu3)
    assert p["rho_nu"] > 1e-5
    x4 = x.copy()
    x4[-1] = qp.meta["u"][-1] + 0.5                 # break an upper bound
    _, p = kkt.rel_kkt(qp, x4, lam, nu)
    assert p["rho_p"] > 1e-3


# --- P3 KKT invariant ------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 5, 11])
def test_oracle_reaches_kkt_tolerance_small_workload(seed):
    qp = synth.gaussian_qp(seed, 200, 50, 100)
    r = ipm.solve(qp)
    assert r.converged and r.rel_kkt <= 1e-10
    assert np.all(r.s > 0) and np.all(r.nu > 0)
    # strict convexity: objective below any feasible point's, here x0 from the generator
    assert r.obj <= kkt.objective(qp, qp.x0) + 1e-9


# --- P4 exact reformulation (Sec. 4.1) ------------------------------------------
def _state(qp, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(qp.n)
    lam = rng.standard_normal(qp.m1)
    nu = rng.uniform(0.1, 2.0, qp.m2)
    s = rng.uniform(0.1, 2.0, qp.m2)
    return x, lam, nu, s


@pytest.mark.parametrize("n,m1,m2", [(12, 4, 9), (20, 15, 30), (16, 1, 16), (10, 10, 6)])
def test_reduced_newton_step_equals_full_system(n, m1, m2):
    qp = synth.gaussian_qp(n + m1 + m2, n, m1, m2)
    x, lam, nu, s = _state(qp, 3)
    mu = s @ nu / m2
    rc = s * nu - 0.3 * mu
    red = reduced.reduced_newton_step(qp, x, lam, nu, s, rc)
    K = ipm.newton_matrix(qp, nu, s)
    rhs = -np.concatenate([qp.H @ x + qp.c - qp.A.T @ lam - qp.C.T @ nu, qp.A @ x - qp.b,
                           qp.C @ x - qp.d - s, rc])
    full = np.linalg.solve(K, rhs)
    red_v = np.concatenate(red)
    assert np.max(np.abs(red_v - full)) <= 1e-9 * (1 + np.max(np.abs(full)))


@pytest.mark.parametrize("n,m1,m2", [(12, 4, 9), (20, 15, 30), (9, 9, 5)])
def test_kf_forms_agree_and_are_spd(n, m1, m2):
    qp = synth.gaussian_qp(99, n, m1, m2)
    dvec = synth.log_uniform(1, m2, 1e-3, 1e3)
    K1 = reduced.kf_explicit(qp, dvec)
    K2 = reduced.kf_from_k0(qp, dvec)
    K3 = reduced.kf_schur_form(qp, dvec)
    sc = np.max(np.abs(K1))
    assert np.max(np.abs(K1 - K2)) <= 1e-11 * sc
    assert np.max(np.abs(K1 - K3)) <= 1e-9 * sc
    assert np.min(np.linalg.eigvalsh(K1)) > 0
    # matrix-free product of the implicit form
    p = np.random.default_rng(0).standard_normal(m2)
    assert np.max(np.abs(reduced.kf_apply(qp, dvec, p) - K1 @ p)) <= 1e-10 * sc * np.max(np.abs(p))


def test_m1_equals_n_gives_kf_equal_D():
    # with A square and nonsingular the feasible set is a point: [C 0]F^{-1}[C^T;0] = 0
    qp = synth.gaussian_qp(4, 8, 8, 5)
    dvec = synth.log_uniform(2, 5, 1e-2, 1e2)
    K = reduced.kf_explicit(qp, dvec)
    assert np.max(np.abs(K - np.diag(dvec))) <= 1e-10 * np.max(dvec)


def test_inertia_of_F():
    qp = synth.gaussian_qp(5, 15, 6, 4)
    w = np.linalg.eigvalsh(reduced.F_matrix(qp))
    assert np.sum(w < 0) == 15 and np.sum(w > 0) == 6


def test_rank_lemmas():
    qp = synth.gaussian_qp(6, 14, 5, 3)
    Hb = reduced.hbar_a(qp)
    sv1 = np.linalg.svd(Hb, compute_uv=False)
    sv2 = np.linalg.svd(qp.H - Hb, compute_uv=False)
    assert np.sum(sv1 > 1e-9 * sv1[0]) <= 5
    assert np.sum(sv2 > 1e-9 * sv2[0]) <= 14 - 5


def test_simple_bounds_ph_is_D_plus_Hinv():
    qp = synth.syqp(1, 12, 4)
    dvec = synth.log_uniform(3, 12, 1e-2, 1e2)
    assert np.allclose(reduced.P_H(qp, dvec), np.diag(dvec) + np.linalg.inv(qp.H), rtol=1e-9, atol=1e-9)


def test_diag_ph_equals_exact_ph_for_diagonal_H():
    """With diagonal H the PH-KF preconditioner of Sec. 5.2 is eq. preconditioner-2 itself."""
    qp = synth.gaussian_qp(5, 14, 4, 9)
    qp.H = np.diag(np.linspace(0.5, 3.0, 14))
    dvec = synth.log_uniform(4, 9, 1e-2, 1e2)
    assert np.allclose(reduced.P_H_diag(qp, dvec), reduced.P_H(qp, dvec), rtol=1e-12, atol=1e-12)


def test_diag_ph_entries_by_definition():
    """Entry (i, j) of C diag(H)^{-1} C^T is sum_k C_ik C_jk / H_kk (loops on a tiny case)."""
    qp = synth.gaussian_qp(6, 5, 2, 4)
    T = reduced.ph_T_diag(qp)
    for i in range(4):
        for j in range(4):
            ref = sum(qp.C[i, k] * qp.C[j, k] / qp.H[k, k] for k in range(5))
            assert abs(T[i, j] - ref) <= 1e-13 * max(1.0, abs(ref))


# --- P6 spectral theorems -------------------------------------------------------
@pytest.mark.parametrize("n,m1,m2", [(20, 15, 30), (24, 6, 30), (30, 10, 12), (16, 1, 40), (20, 19, 25)])
def test_preconditioned_spectra(n, m1, m2):
    qp = synth.gaussian_qp(n * m1 + m2, n, m1, m2)
    dvec = synth.log_uniform(7, m2, 1e-2, 1e2)
    K = reduced.kf_explicit(qp, dvec)
    eL = reduced.preconditioned_eigs(K, reduced.P_L(dvec))
    eH = reduced.preconditioned_eigs(K, reduced.P_H(qp, dvec))
    tol = 1e-8
    assert np.sum(np.abs(eL - 1) > tol) <= min(m2, n - m1)          # Theorem thm1
    assert np.sum(np.abs(eH - 1) > tol) <= min(m2, m1)              # Theorem thm2
    assert np.min(eL) >= 1 - 1e-9                                    # I + X, X PSD
    assert np.min(eH) > 0 and np.max(eH) <= 1 + 1e-9                 # I - Y, 0 < ... <= 1
    # the bounds are attained generically, so the count is not vacuous
    assert np.sum(np.abs(eL - 1) > tol) == min(m2, n - m1)
    assert np.sum(np.abs(eH - 1) > tol) == min(m2, m1)


# --- P7 CG iteration corollaries -------------------------------------------------
@pytest.mark.parametrize("n,m1,m2,which", [(30, 26, 40, "L"), (30, 3, 40, "H"), (24, 20, 24, "L"),
                                           (24, 2, 30, "H")])
def test_cg_iteration_bounds(n, m1, m2, which):
    qp = synth.gaussian_qp(n + 100 * m1 + m2, n, m1, m2)
    dvec = synth.log_uniform(11, m2, 1e-2, 1e2)
    K = reduced.kf_explicit(qp, dvec)
    b = np.random.default_rng(1).standard_normal(m2)
    if which == "L":
        P = reduced.P_L(dvec)
        bound = min(m2, n - m1)
    else:
        P = reduced.P_H(qp, dvec)
        bound = min(m2, m1)
    cf = sla.cho_factor(P)
    # Corollaries cor:cg1 / cor:cg2: exact arithmetic terminates after bound + 1
    # steps; in float64 the residual collapses there (to rounding level), while
    # one step earlier it is still of the order of the right-hand side.
    x, k, h = reduced.pcg(lambda v: K @ v, b, lambda r: sla.cho_solve(cf, r), 0.0, bound + 1)
    assert k == bound + 1
    assert h[bound + 1] <= 1e-6 * h[0]
    assert h[bound - 1] >= 1e-3 * h[0]
    xd = sla.cho_solve(sla.cho_factor(K), b)
    assert np.linalg.norm(x - xd) <= 1e-5 * np.linalg.norm(xd)


def test_cg_special_cases():
    # m1 = n: K_F = D, so P_L CG converges in one step
    qp = synth.gaussian_qp(8, 10, 10, 7)
    dvec = synth.log_uniform(2, 7, 1e-2, 1e2)
    K = reduced.kf_explicit(qp, dvec)
    b = np.ones(7)
    _, k, h = reduced.pcg(lambda v: K @ v, b, lambda r: r / dvec, 0.0, 1)
    assert h[1] <= 1e-12 * h[0]
    # m1 = 1: P_H CG needs at most two steps
    qp = synth.gaussian_qp(9, 20, 1, 25)
    dvec = synth.log_uniform(3, 25, 1e-2, 1e2)
    K = reduced.kf_explicit(qp, dvec)
    cf = sla.cho_factor(reduced.P_H(qp, dvec))
    _, k, h = reduced.pcg(lambda v: K @ v, np.ones(25), lambda r: sla.cho_solve(cf, r), 0.0, 2)
    assert h[2] <= 1e-6 * h[0] and h[1] >= 1e-3 * h[0]


# --- mutation tests: plant a mistake in the oracle, a pin must catch it ----------
def test_mutation_sign_error_in_newton_matrix_is_caught(monkeypatch):
    orig = ipm.newton_matrix

    def bad(qp, nu, s):
        K = orig(qp, nu, s)
        n, m1 = qp.n, qp.m1
        K[:n, n:n + m1] *= -1.0                      # wrong sign on -A^T
        return K
    monkeypatch.setattr(ipm, "newton_matrix", bad)
    qp = synth.tiny_qp(0, 5, 2, 8)
    xb, *_ = bruteforce.solve(qp)
    r = ipm.solve(qp, tol=1e-12, max_iter=60)
    assert (not r.converged) or np.max(np.abs(r.x - xb)) > 1e-6


def test_mutation_dropped_term_in_kf_is_caught(monkeypatch):
    qp = synth.gaussian_qp(1, 20, 15, 30)
    dvec = synth.log_uniform(7, 30, 1e-2, 1e2)

    def bad(qp_, d_):                                # dropped D term
        return reduced.kf_from_k0(qp_, d_) - np.diag(d_)
    assert np.max(np.abs(bad(qp, dvec) - reduced.kf_explicit(qp, dvec))) > 1e-3
    # the spectral pin fails for a transposed C in P_H
    K = reduced.kf_explicit(qp, dvec)
    T_bad = qp.C @ np.linalg.solve(qp.H, qp.C.T) * 0.5
    eH = reduced.preconditioned_eigs(K, np.diag(dvec) + T_bad)
    assert np.sum(np.abs(eH - 1) > 1e-8) > min(30, 15)


def test_mutation_wrong_corrector_is_caught(monkeypatch):
    # a corrector that forgets the second-order term still converges but the
    # brute-force pin is met; one that flips sigma's sign must not converge to it
    real_solve = ipm.solve
    qp = synth.tiny_qp(2, 6, 3, 10)
    xb, *_ = bruteforce.solve(qp)
    orig = ipm.max_step
    monkeypatch.setattr(ipm, "max_step", lambda v, dv: 2.0 * orig(v, dv))   # overshoots the boundary
    r = real_solve(qp, tol=1e-12, max_iter=60, check=False)
    bad = (not r.converged) or np.max(np.abs(r.x - xb)) > 1e-6 or np.any(r.s <= 0) or np.any(r.nu <= 0)
    assert bad

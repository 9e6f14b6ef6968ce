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


def test_mutation_overshooting_step_rule_is_caught(monkeypatch):
    # a fraction-to-boundary rule that steps twice as far as the boundary allows
    # leaves the interior: the brute-force pin or the positivity invariant fails
    real_solve = ipm.solve
    qp = synth.tiny_qp(2, 6, 3, 10)
    xb, *_ = bruteforce.solve(qp)
    orig = ipm.max_step
    monkeypatch.setattr(ipm, "max_step", lambda v, dv: 2.0 * orig(v, dv))   # overshoots the boundary
    r = real_solve(qp, tol=1e-12, max_iter=60, check=False)
    bad = (not r.converged) or np.max(np.abs(r.x - xb)) > 1e-6 or np.any(r.s <= 0) or np.any(r.nu <= 0)
    assert bad


@pytest.mark.parametrize("mutation", ["no_second_order_term", "sigma_linear", "sigma_sign"])
def test_mutation_wrong_corrector_is_caught(monkeypatch, mutation):
    """A corrector or centering rule other than Mehrotra's is caught by the scalar recurrence pin."""
    if mutation == "no_second_order_term":
        monkeypatch.setattr(ipm, "corrector_rc", lambda s, nu, dsa, dna, sg, mu: s * nu - sg * mu)
    elif mutation == "sigma_linear":
        monkeypatch.setattr(ipm, "centering", lambda mu, mu_aff: mu_aff / mu)
    else:
        orig = ipm.corrector_rc
        monkeypatch.setattr(ipm, "corrector_rc", lambda s, nu, dsa, dna, sg, mu: orig(s, nu, dsa, dna, -sg, mu))
    with pytest.raises(AssertionError):
        for case in _SCALAR_CASES:
            _check_scalar_recurrence(*case)


# --- validate: the assumptions of Sec. 1 are enforced -----------------------------
def _qp_with(qp, **kw):
    q = synth.QP(*(np.array(a, copy=True) for a in qp.arrays()))
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def test_validate_accepts_the_generator_instances():
    ipm.validate(synth.gaussian_qp(1, 30, 10, 20))
    ipm.validate(synth.gaussian_qp(2, 12, 12, 5))       # m1 = n is allowed (Sec. 1)
    ipm.validate(synth.illcond_qp(3, 32, 4, 32))


def test_validate_rejects_asymmetric_H_at_its_tolerance():
    qp = synth.gaussian_qp(4, 20, 6, 10)
    scale = max(1.0, np.linalg.norm(qp.H))
    # one off-diagonal entry perturbed by delta gives ||H - H^T||_F = sqrt(2) delta
    for delta, ok in [(0.5e-14 * scale, True), (1.0e-14 * scale, False), (1e-6, False)]:
        H = qp.H.copy()
        H[0, 3] += delta
        q = _qp_with(qp, H=H)
        if ok:
            ipm.validate(q)
        else:
            with pytest.raises(ipm.OracleInputError, match="symmetric"):
                ipm.validate(q)


@pytest.mark.parametrize("lam_min", [-1e-3, -1.0, -1e-8])
def test_validate_rejects_H_that_is_not_positive_definite(lam_min):
    qp = synth.gaussian_qp(5, 16, 4, 8)
    rng = np.random.default_rng(0)
    U, _ = np.linalg.qr(rng.standard_normal((16, 16)))
    w = np.linspace(0.5, 2.0, 16)
    w[3] = lam_min
    H = (U * w) @ U.T
    H = 0.5 * (H + H.T)
    with pytest.raises(ipm.OracleInputError, match="positive definite"):
        ipm.validate(_qp_with(qp, H=H))


def test_validate_rejects_rank_deficient_A_at_the_svd_threshold():
    """rank A = m1 is tested with sigma_min > max(m1, n) eps sigma_max; both sides of it."""
    n, m1 = 20, 6
    qp = synth.gaussian_qp(6, n, m1, 10)
    rng = np.random.default_rng(1)
    U, _ = np.linalg.qr(rng.standard_normal((m1, m1)))
    V, _ = np.linalg.qr(rng.standard_normal((n, m1)))
    tol = max(m1, n) * np.finfo(float).eps
    for factor, ok in [(4.0, True), (0.25, False)]:
        sv = np.linspace(1.0, 0.5, m1)
        sv[-1] = factor * tol * sv[0]
        A = (U * sv) @ V.T
        q = _qp_with(qp, A=A)
        if ok:
            ipm.validate(q)
        else:
            with pytest.raises(ipm.OracleInputError, match="rank"):
                ipm.validate(q)
    # an exactly dependent row
    A = qp.A.copy()
    A[2] = A[0] - 3.0 * A[1]
    with pytest.raises(ipm.OracleInputError, match="rank"):
        ipm.validate(_qp_with(qp, A=A))


def test_validate_rejects_bad_sizes():
    qp = synth.gaussian_qp(7, 8, 3, 5)
    wide = synth.gaussian_qp(7, 8, 9, 5)                 # m1 > n
    with pytest.raises(ipm.OracleInputError, match="m1"):
        ipm.validate(_qp_with(qp, A=wide.A, b=wide.b))
    with pytest.raises(ipm.OracleInputError, match="m1"):
        ipm.validate(_qp_with(qp, A=np.zeros((0, 8)), b=np.zeros(0)))


# --- dual objective: the Lagrangian of eq. lagrangian at a stationary point ------
def test_dual_objective_is_the_lagrangian_at_a_stationary_point():
    rng = np.random.default_rng(3)
    qp = synth.gaussian_qp(8, 25, 7, 15)
    for _ in range(5):
        x = rng.standard_normal(25)
        lam = rng.standard_normal(7)
        nu = rng.uniform(0.0, 2.0, 15)
        # choose c so that grad_x L = H x + c - A^T lam - C^T nu = 0 (Sec. 2)
        q = _qp_with(qp, c=qp.A.T @ lam + qp.C.T @ nu - qp.H @ x,
                     b=rng.standard_normal(7), d=rng.standard_normal(15))
        L = (0.5 * x @ q.H @ x + x @ q.c - lam @ (q.A @ x - q.b) - nu @ (q.C @ x - q.d))
        assert abs(kkt.dual_objective(q, x, lam, nu) - L) <= 1e-11 * (1 + abs(L))
        # and primal minus dual is lam^T (A x - b) + nu^T (C x - d)
        gap = kkt.objective(q, x) - kkt.dual_objective(q, x, lam, nu)
        assert abs(gap - (lam @ (q.A @ x - q.b) + nu @ (q.C @ x - q.d))) <= 1e-10 * (1 + abs(gap))


def test_dual_objective_strong_and_weak_duality():
    qp = synth.box_qp(2, 12, 4)
    x, lam, nu = boxqp.solve(qp)
    # strong duality at the closed-form optimum
    f = kkt.objective(qp, x)
    assert abs(kkt.dual_objective(qp, x, lam, nu) - f) <= 1e-13 * (1 + abs(f))
    # weak duality: a dual-feasible point (stationary, nu >= 0) bounds every feasible objective
    rng = np.random.default_rng(5)
    nf = qp.n - qp.m1
    for _ in range(5):
        xs = x.copy()
        xs[qp.m1:] = rng.uniform(qp.meta["l"], qp.meta["u"])       # another feasible point
        nu2 = nu + rng.uniform(0.0, 0.3, 2 * nf)
        lam2 = qp.H[:qp.m1, :qp.m1] @ xs[:qp.m1] + qp.c[:qp.m1]
        # the x that makes (lam2, nu2) stationary: H x = A^T lam2 + C^T nu2 - c
        xd = np.linalg.solve(qp.H, qp.A.T @ lam2 + qp.C.T @ nu2 - qp.c)
        assert kkt.dual_objective(qp, xd, lam2, nu2) <= kkt.objective(qp, xs) + 1e-12


# --- Newton residuals: signs of eq. rhs-KKT4 against eq. sym-indef-KKT ----------
@pytest.mark.parametrize("n,m1,m2", [(10, 3, 8), (15, 15, 6)])
def test_newton_residuals_vanish_after_a_full_newton_step(n, m1, m2):
    """Rows 1-3 of eq. sym-indef-KKT are linear, so a full step zeroes their residuals."""
    qp = synth.gaussian_qp(n + m2, n, m1, m2)
    x, lam, nu, s = _state(qp, 9)
    mu = s @ nu / m2
    r_g, r_e, r_i = kkt.newton_residuals(qp, x, lam, nu, s)
    r_c = s * nu - 0.2 * mu
    # coefficient matrix of eq. sym-indef-KKT, entered from the paper
    N = n + m1 + 2 * m2
    K = np.zeros((N, N))
    i1, i2, i3 = n, n + m1, n + m1 + m2
    K[:i1, :i1] = -qp.H
    K[:i1, i1:i2] = qp.A.T
    K[:i1, i2:i3] = qp.C.T
    K[i1:i2, :i1] = qp.A
    K[i2:i3, :i1] = qp.C
    K[i2:i3, i3:] = -np.eye(m2)
    K[i3:, i2:i3] = np.diag(s)
    K[i3:, i3:] = np.diag(nu)
    step = np.linalg.solve(K, -np.concatenate([r_g, r_e, r_i, r_c]))
    dx, dl, dn, ds = np.split(step, [i1, i2, i3])
    g2, e2, i2_ = kkt.newton_residuals(qp, x + dx, lam + dl, nu + dn, s + ds)
    for before, after in [(r_g, g2), (r_e, e2), (r_i, i2_)]:
        assert np.max(np.abs(after)) <= 1e-9 * (1 + np.max(np.abs(before)))
    # r_g is minus the gradient of the Lagrangian of eq. lagrangian
    assert np.allclose(r_g, -(qp.H @ x + qp.c - qp.A.T @ lam - qp.C.T @ nu), rtol=0, atol=1e-12)
    # and the oracle's eq. nonsym-indef-KKT step is the same step
    full = np.linalg.solve(ipm.newton_matrix(qp, nu, s), -np.concatenate([-r_g, r_e, r_i, r_c]))
    assert np.max(np.abs(full - step)) <= 1e-9 * (1 + np.max(np.abs(step)))


# --- Mehrotra predictor-corrector against a hand-eliminated scalar recurrence ----
# n = 2, m1 = 1, m2 = 1: A = [1 0] fixes x_1 = beta, C = [0 1] bounds x_2 >= delta.
# The Newton system of eq. nonsym-indef-KKT then reduces by hand to scalars:
#   h2 dx - dnu = -r_d,  dx - ds = -r_i,  s dnu + nu ds = -r_c
#   => dx = -(r_c + s r_d + nu r_i) / (s h2 + nu),  dnu = h2 dx + r_d,  ds = dx + r_i.
_SCALAR_CASES = [
    # h1, h2, c1, c2, beta, delta: bound active at the optimum (x2* = delta, nu* = h2 delta + c2 > 0)
    (2.0, 1.0, 0.5, 2.0, 1.5, 0.5),
    # bound inactive (x2* = -c2/h2 > delta, nu* = 0)
    (1.0, 0.5, -1.0, -1.5, -0.5, 0.5),
    # start feasible, strongly active bound
    (3.0, 4.0, 0.0, 10.0, 2.0, -3.0),
]


def _scalar_qp(h1, h2, c1, c2, beta, delta):
    return synth.QP(np.diag([h1, h2]), np.array([c1, c2]), np.array([[1.0, 0.0]]), np.array([beta]),
                    np.array([[0.0, 1.0]]), np.array([delta]))


def _check_scalar_recurrence(h1, h2, c1, c2, beta, delta, tau=0.995, iters=8):
    qp = _scalar_qp(h1, h2, c1, c2, beta, delta)
    r = ipm.solve(qp, tol=1e-13, max_iter=60)

    def step_to_boundary(v, dv):
        return -v / dv if dv < 0 else np.inf

    def newton(x2, nu, s, rc):
        r_d = h2 * x2 + c2 - nu
        r_i = x2 - delta - s
        dx = -(rc + s * r_d + nu * r_i) / (s * h2 + nu)
        return dx, h2 * dx + r_d, dx + r_i

    # initial point: the equality-only QP, s0 = max(C x0 - d, 1), nu0 = 1
    x2 = -c2 / h2
    s, nu = max(x2 - delta, 1.0), 1.0
    for k in range(min(iters, len(r.history))):
        mu = s * nu
        dxa, dna, dsa = newton(x2, nu, s, s * nu)
        a_aff = min(1.0, step_to_boundary(s, dsa), step_to_boundary(nu, dna))
        sigma = ((s + a_aff * dsa) * (nu + a_aff * dna) / mu) ** 3
        dx, dn, ds = newton(x2, nu, s, s * nu + dsa * dna - sigma * mu)
        alpha = min(1.0, tau * min(step_to_boundary(s, ds), step_to_boundary(nu, dn)))
        h = r.history[k]
        assert abs(h["mu"] - mu) <= 1e-9 * mu, (k, h["mu"], mu)
        assert abs(h["sigma"] - sigma) <= 1e-7 * max(sigma, 1e-12), (k, h["sigma"], sigma)
        assert abs(h["alpha"] - alpha) <= 1e-9, (k, h["alpha"], alpha)
        x2, nu, s = x2 + alpha * dx, nu + alpha * dn, s + alpha * ds
    # the limit is the closed-form minimizer of the one-bound problem
    x2_star = max(-c2 / h2, delta)
    assert r.converged
    assert abs(r.x[0] - beta) <= 1e-12 * (1 + abs(beta))
    assert abs(r.x[1] - x2_star) <= 1e-9 * (1 + abs(x2_star))
    assert abs(r.lam[0] - (h1 * beta + c1)) <= 1e-9 * (1 + abs(h1 * beta + c1))
    assert abs(r.nu[0] - max(h2 * delta + c2, 0.0)) <= 1e-9 * (1 + abs(c2))


@pytest.mark.parametrize("case", _SCALAR_CASES)
def test_mehrotra_iterates_match_scalar_recurrence(case):
    _check_scalar_recurrence(*case)


@pytest.mark.parametrize("seed,n,m1", [(3, 4, 1), (4, 5, 2)])
def test_bruteforce_matches_closed_form_box_qp(seed, n, m1):
    """The two independent pins agree with each other on the box QP."""
    qp = synth.box_qp(seed, n, m1)
    xc, lc, nc = boxqp.solve(qp)
    xb, lb, nb, _ = bruteforce.solve(qp)
    assert np.max(np.abs(xb - xc)) <= 1e-12
    assert np.max(np.abs(lb - lc)) <= 1e-12
    assert np.max(np.abs(nb - nc)) <= 1e-12

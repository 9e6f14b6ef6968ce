"""CPU oracle for the preconditioned implicit-PCG interior point method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
execute this package; only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP path: it is plain float64
NumPy/SciPy, written from the paper (Karim & Solomonik, "Efficient
Preconditioners for Interior Point Methods via a new Schur Complement-Based
Strategy").

Modules
-------
kkt         KKT residuals of eq. qp and the slack-free relative KKT score.
ipm         Full-system primal-dual IPM: each Newton step solves the unreduced
            4 x 4 block system of eq. nonsym-indef-KKT by dense LU.  It never forms
            the reduced matrix, so it checks the reformulation instead of
            repeating it.
reduced     The reformulation written out on explicit matrices: F (eq. f-def),
            K_F and r_nu (eq. ineq-const-reduced), the recovery of eq.
            schur-delta-x, the block-inverse form of eq. schur-R, the
            preconditioners P_L and P_H (eqs. preconditioner-1/-2), preconditioned
            spectra (Theorems thm1/thm2) and a textbook PCG (Sec. 6 protocol).
bruteforce  Active-set enumeration for tiny QPs (a pin for ipm).
boxqp       Closed-form minimizer of a separable box-constrained QP (a pin).

Every function states the passage it follows.  Pins that tie these functions to
facts other than themselves live in tests/test_oracle_*.py.
"""
from . import kkt, ipm, reduced, bruteforce, boxqp  # noqa: F401

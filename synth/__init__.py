"""Seeded synthetic inputs shared by the oracle, the GPU tests and the benchmark.

This module only draws random data and assembles problem instances of

    minimize 1/2 x^T H x + c^T x   s.t.  A x = b,  C x >= d          (eq. qp, Sec. 1)

It contains none of the solver's arithmetic: no factorization, no reduced
system, no Newton step.  Every array is float64, C-contiguous, row-major.

Generators
----------
gaussian_qp(seed, n, m1, m2)
    Dense Gaussian instance.  ``numpy.random.default_rng(seed)`` (PCG64) draws, in
    this fixed order: Q (n x n), c (n), A (m1 x n), C (m2 x n), x0 (n), s (m2).
    Q, c, A, C, x0 are N(0, 1); s is U(0.1, 1).  H = Q^T Q / n + 1e-2 I,
    symmetrized; b = A x0 and d = C x0 - s, so x0 is strictly feasible.
illcond_qp(seed, n, m1, m2)
    Same draws and order, but the n x n Gaussian block becomes a Haar-orthogonal
    U (QR with the signs of diag(R) folded in) and H = U diag(logspace(-4, 2, n)) U^T.
box_qp(seed, n, m1)
    Diagonal H, A = [I_m1 0], two-sided box bounds on the free coordinates
    (C = [0 I; 0 -I]).  Its minimizer has a closed form, used as a test pin.
batch_sizes / serving_stream
    Size mixes of the batched and streamed workloads.
shared_family(seed, n, m1, m2, k)
    k QPs with one H, A, C and their own c, b, d (QPs that share the K0 factor).
syqp(seed, n, m1)
    The paper's synthetic family SyQP^n_{m1} (Sec. 6.1): block-diagonal H made of
    4 x 4 blocks M^T M with M ~ U[0, 1], banded A with U[0, 1) entries, C = I, d = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "QP", "gaussian_qp", "illcond_qp", "box_qp", "syqp", "tiny_qp",
    "batch_sizes", "batch_sample", "large_batch_sizes", "serving_stream", "log_uniform", "workload",
    "shared_family",
]


@dataclass
class QP:
    """One problem instance, all arrays float64 row-major."""
    H: np.ndarray
    c: np.ndarray
    A: np.ndarray
    b: np.ndarray
    C: np.ndarray
    d: np.ndarray
    x0: np.ndarray | None = None          # a strictly feasible point, when known
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.H.shape[0]

    @property
    def m1(self) -> int:
        return self.A.shape[0]

    @property
    def m2(self) -> int:
        return self.C.shape[0]

    def arrays(self):
        return self.H, self.c, self.A, self.b, self.C, self.d


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _finish(H, c, A, C, x0, s, meta):
    H = 0.5 * (H + H.T)
    b = A @ x0
    d = C @ x0 - s
    return QP(_c(H), _c(c), _c(A), _c(b), _c(C), _c(d), _c(x0), meta)


def gaussian_qp(seed: int, n: int, m1: int, m2: int) -> QP:
    """Dense Gaussian QP with H = Q^T Q / n + 1e-2 I (see module docstring)."""
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    c = rng.standard_normal(n)
    A = rng.standard_normal((m1, n))
    C = rng.standard_normal((m2, n))
    x0 = rng.standard_normal(n)
    s = rng.uniform(0.1, 1.0, m2)
    H = Q.T @ Q / n + 1e-2 * np.eye(n)
    return _finish(H, c, A, C, x0, s,
                   dict(kind="gaussian", seed=seed, n=n, m1=m1, m2=m2))


def illcond_qp(seed: int, n: int, m1: int, m2: int) -> QP:
    """Gaussian QP whose Hessian has eigenvalues logspaced 1e-4..1e2 in a Haar basis."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    c = rng.standard_normal(n)
    A = rng.standard_normal((m1, n))
    C = rng.standard_normal((m2, n))
    x0 = rng.standard_normal(n)
    s = rng.uniform(0.1, 1.0, m2)
    U, R = np.linalg.qr(G)
    U = U * np.sign(np.diag(R))[None, :]
    lam = np.logspace(-4.0, 2.0, n)
    H = (U * lam[None, :]) @ U.T
    return _finish(H, c, A, C, x0, s,
                   dict(kind="illcond", seed=seed, n=n, m1=m1, m2=m2))


def tiny_qp(seed: int, n: int, m1: int, m2: int) -> QP:
    """Alias of gaussian_qp for the brute-force sizes (n <= 6)."""
    return gaussian_qp(seed, n, m1, m2)


def box_qp(seed: int, n: int, m1: int) -> QP:
    """Separable QP: H = diag(h), A = [I_m1 0], l <= x_j <= u_j for j >= m1.

    C = [[0, I], [0, -I]] and d = [l; -u] (so m2 = 2 (n - m1)).  Centers
    -c_j / h_j are spread so that some coordinates end up at l, some at u and
    some strictly inside.
    """
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.5, 2.0, n)
    c = rng.standard_normal(n) * 2.0
    b = rng.standard_normal(m1)
    nf = n - m1
    l = rng.uniform(-1.0, -0.2, nf)
    u = rng.uniform(0.2, 1.0, nf)
    H = np.diag(h)
    A = np.zeros((m1, n))
    A[:, :m1] = np.eye(m1)
    C = np.zeros((2 * nf, n))
    C[:nf, m1:] = np.eye(nf)
    C[nf:, m1:] = -np.eye(nf)
    d = np.concatenate([l, -u])
    x0 = np.concatenate([b, 0.5 * (l + u)])
    return QP(_c(H), _c(c), _c(A), _c(b), _c(C), _c(d), _c(x0),
              dict(kind="box", seed=seed, n=n, m1=m1, m2=2 * nf, h=h, l=l, u=u))


def syqp(seed: int, n: int, m1: int, band: int = 3, H_seed: int | None = None) -> QP:
    """SyQP^n_{m1}: block-diagonal 4x4 M^T M Hessian, banded A, x >= 0 (Sec. 6.1).

    ``H_seed`` lets a family share one Hessian across m1, as the paper does.
    A row i has nonzeros in columns i .. i + band (clipped), U[0, 1) entries, and a
    unit added on its leading entry so that A keeps full row rank.  b = A x0 for an
    x0 ~ U(0.5, 1.5) > 0 (strictly feasible); c ~ U[0, 1).
    """
    rng_h = np.random.default_rng(seed if H_seed is None else H_seed)
    H = np.zeros((n, n))
    for k in range(0, n, 4):
        w = min(4, n - k)
        M = rng_h.uniform(0.0, 1.0, (w, w))
        H[k:k + w, k:k + w] = M.T @ M
    H += 1e-8 * np.eye(n)          # keep the random blocks safely nonsingular
    rng = np.random.default_rng(seed + 7919)
    A = np.zeros((m1, n))
    for i in range(m1):
        j0 = min(i, n - 1)
        j1 = min(n, j0 + band + 1)
        A[i, j0:j1] = rng.uniform(0.0, 1.0, j1 - j0)
        A[i, j0] += 1.0
    c = rng.uniform(0.0, 1.0, n)
    x0 = rng.uniform(0.5, 1.5, n)
    C = np.eye(n)
    d = np.zeros(n)
    H = 0.5 * (H + H.T)
    return QP(_c(H), _c(c), _c(A), _c(A @ x0), _c(C), _c(d), _c(x0),
              dict(kind="syqp", seed=seed, n=n, m1=m1, m2=n))


def shared_family(seed: int, n: int, m1: int, m2: int, k: int, base=None) -> list:
    """k QPs sharing H, A and C (those of ``base``, default gaussian_qp(seed, n, m1, m2)).

    QP j draws, from ``default_rng(seed + 1 + j)`` in this order, c_j ~ N(0, 1),
    x0_j ~ N(0, 1) and s_j ~ U(0.1, 1); b_j = A x0_j and d_j = C x0_j - s_j, so
    x0_j is strictly feasible for QP j.
    """
    base = gaussian_qp(seed, n, m1, m2) if base is None else base
    out = []
    for j in range(k):
        rng = np.random.default_rng(seed + 1 + j)
        c = rng.standard_normal(base.n)
        x0 = rng.standard_normal(base.n)
        s = rng.uniform(0.1, 1.0, base.m2)
        out.append(QP(base.H, _c(c), base.A, _c(base.A @ x0), base.C, _c(base.C @ x0 - s), _c(x0),
                      dict(kind="shared", seed=seed, j=j, n=base.n, m1=base.m1, m2=base.m2)))
    return out


def log_uniform(seed: int, size: int, lo: float, hi: float) -> np.ndarray:
    """Positive vector with log10 entries uniform in [log10 lo, log10 hi]."""
    rng = np.random.default_rng(seed)
    return _c(10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size))


def batch_sizes(count: int = 512, seed: int = 1000):
    """Sizes of the batched workload: n ~ U{64..1024}, m1 = n // 4, m2 = n // 2.

    Returns a list of (seed_i, n, m1, m2) with seed_i = seed + i; the sizes come
    from their own stream ``default_rng(seed)`` so the per-instance draws keep the
    Q, c, A, C, x0, s order.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(64, 1025, size=count)
    return [(seed + i, int(n), int(n) // 4, int(n) // 2) for i, n in enumerate(ns)]


def batch_sample(count: int = 24, top: int = 8, total: int = 512, seed: int = 1000):
    """A fixed sample of the batched workload's draw batch_sizes(total, seed).

    The ``top`` largest QPs of the draw (its n >= 1008 end) and ``count - top``
    others evenly spaced in the order of n, so the sample spans the whole size
    range.  Returns (seed_i, n, m1, m2) tuples in draw order.
    """
    sizes = batch_sizes(total, seed)
    ns = np.array([sz[1] for sz in sizes])
    order = np.argsort(ns, kind="stable")
    rest = order[:-top]
    pick = rest[np.linspace(0, len(rest) - 1, count - top).round().astype(int)]
    return [sizes[i] for i in sorted(set(order[-top:].tolist()) | set(pick.tolist()))]


def large_batch_sizes():
    """QPs of the batched workload's shape (m1 = n/4, m2 = n/2) above its n <= 1024
    range, at n = 1500, 2500 and 4000 (the largest sizes of the streamed mix)."""
    return [(7001, 1500, 375, 750), (7002, 2500, 625, 1250), (7003, 4000, 1000, 2000)]


def serving_stream(count: int, seed: int = 5000, base: int = 10 ** 6,
                   n_lo: int = 128, n_hi: int = 4096):
    """Request mix of the streamed workload.

    n = round(exp(U(ln n_lo, ln n_hi))), m1 = floor(n U(1/8, 1/2)) (at least 1),
    m2 = floor(n U(1/2, 1)); request i uses instance seed base + i.  Returns a list
    of (seed_i, n, m1, m2).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m1 = max(1, int(math.floor(n * rng.uniform(1 / 8, 1 / 2))))
        m2 = max(1, int(math.floor(n * rng.uniform(1 / 2, 1))))
        out.append((base + i, n, m1, m2))
    return out


# Named workloads (dense Gaussian unless stated): small parity case, many
# equalities (low degrees of freedom), few equalities with an ill-conditioned H.
WORKLOADS = {
    "small": dict(gen="gaussian", n=200, m1=50, m2=100, seeds=list(range(16))),
    "lowdof": dict(gen="gaussian", n=4096, m1=3072, m2=2048, seeds=[100, 101, 102]),
    "fewEq": dict(gen="illcond", n=4096, m1=256, m2=4096, seeds=[200, 201, 202]),
}


def workload(name: str, seed: int | None = None, scale: float = 1.0) -> QP:
    """Instance of a named workload; ``scale`` < 1 shrinks every dimension."""
    w = WORKLOADS[name]
    s = w["seeds"][0] if seed is None else seed
    n = max(2, int(round(w["n"] * scale)))
    m1 = max(1, int(round(w["m1"] * scale)))
    m2 = max(1, int(round(w["m2"] * scale)))
    gen = gaussian_qp if w["gen"] == "gaussian" else illcond_qp
    return gen(s, n, m1, m2)

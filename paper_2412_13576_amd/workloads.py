"""Seeded synthetic instance generators.

This module only draws random problem data: the integer program
(min f(x) s.t. Ax = b, l <= x <= u, x integer; Section 1, eq. INLP), the
objective coefficients and the random start arrays.  It holds none of the
method's arithmetic, so both the CPU oracle and the HIP path may use it.

The paper evaluates on QPLIB / MINLPLib instances (Section 4.1.1) with
50-676 variables and 1-13090 constraints and quadratic or polynomial
objectives (Table 1).  Those suites are not available here; the laws below
are synthetic stand-ins with the same kinds of shape, sparsity and
objective.  Every draw uses numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Instance:
    """One integer program  min f(x)  s.t.  Ax = b,  l <= x <= u,  x in Z^n.

    f is either quadratic  f(x) = x^T Q x + c^T x  (Q symmetric), or a
    separable polynomial  f(x) = sum_i sum_k coef[i, k] * x_i^k  (k = 0..deg).
    x0 is the feasible point b was built from.
    """

    name: str
    A: np.ndarray            # (m, n) int64
    b: np.ndarray            # (m,)  int64
    l: np.ndarray            # (n,)  int64
    u: np.ndarray            # (n,)  int64
    x0: np.ndarray           # (n,)  int64, A x0 = b, l <= x0 <= u
    f_kind: str              # "quadratic" | "separable_poly"
    Q: Optional[np.ndarray] = None     # (n, n) float64
    c: Optional[np.ndarray] = None     # (n,)  float64
    coef: Optional[np.ndarray] = None  # (n, deg+1) float64, coef[i, k] multiplies x_i^k
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.A.shape[0])

    @property
    def n(self) -> int:
        return int(self.A.shape[1])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _full_row_rank(A: np.ndarray) -> bool:
    return int(np.linalg.matrix_rank(A.astype(np.float64))) == A.shape[0]


def tiny_instance(seed: int = 1000) -> Instance:
    """The tiny FP64 parity instance: m=2, n=8.

    A iid uniform integers in [-3, 3] (redrawn until rank 2); x0 uniform in
    [-2, 2]^8; b = A x0; l = -5, u = 5; f = x^T Q x + c^T x with Q = M^T M,
    M 8x8 iid uniform integers in [-2, 2], c iid uniform integers in [-5, 5].
    """
    rng = _rng(seed)
    m, n = 2, 8
    while True:
        A = rng.integers(-3, 4, size=(m, n), dtype=np.int64)
        if _full_row_rank(A):
            break
    x0 = rng.integers(-2, 3, size=n, dtype=np.int64)
    M = rng.integers(-2, 3, size=(n, n), dtype=np.int64)
    Q = (M.T @ M).astype(np.float64)
    c = rng.integers(-5, 6, size=n, dtype=np.int64).astype(np.float64)
    return Instance(name=f"tiny_m2_n8_s{seed}", A=A, b=A @ x0,
                    l=np.full(n, -5, np.int64), u=np.full(n, 5, np.int64),
                    x0=x0, f_kind="quadratic", Q=Q, c=c,
                    meta=dict(law="tiny", seed=seed))


def qp_instance(seed: int = 2000, m: int = 20, n: int = 100) -> Instance:
    """QP-shaped instance: m=20, n=100 by default.

    A iid in {-1, 0, 1} with P(nonzero) = 0.3 and +-1 equiprobable; x0
    uniform integers in [-3, 3]; b = A x0; l = -10, u = 10; f nonconvex
    quadratic: Q symmetric with upper triangle (diagonal included) iid
    N(0, 1) mirrored, c iid N(0, 1).
    """
    rng = _rng(seed)
    while True:
        nz = rng.random((m, n)) < 0.3
        sg = np.where(rng.random((m, n)) < 0.5, -1, 1)
        A = (nz * sg).astype(np.int64)
        if _full_row_rank(A):
            break
    x0 = rng.integers(-3, 4, size=n, dtype=np.int64)
    U = np.triu(rng.standard_normal((n, n)))
    Q = U + np.triu(U, 1).T
    c = rng.standard_normal(n)
    return Instance(name=f"qp_m{m}_n{n}_s{seed}", A=A, b=A @ x0,
                    l=np.full(n, -10, np.int64), u=np.full(n, 10, np.int64),
                    x0=x0, f_kind="quadratic", Q=Q, c=c,
                    meta=dict(law="qp", seed=seed))


def quartic_instance(seed: int = 3000, m: int = 50, n: int = 400) -> Instance:
    """Sparse instance with a separable degree-4 objective: m=50, n=400.

    Each row of A has 4 nonzeros in distinct random columns, values uniform
    in {+-1, ..., +-5}; x0 uniform integers in [-3, 3]; l = -20, u = 20;
    f(x) = sum_i a_i x_i^4 + b_i x_i^3 + c_i x_i^2 with a_i ~ U(0.1, 1),
    b_i, c_i ~ N(0, 1).
    """
    rng = _rng(seed)
    while True:
        A = np.zeros((m, n), np.int64)
        for i in range(m):
            cols = rng.choice(n, size=4, replace=False)
            mag = rng.integers(1, 6, size=4)
            sg = np.where(rng.random(4) < 0.5, -1, 1)
            A[i, cols] = mag * sg
        if _full_row_rank(A):
            break
    x0 = rng.integers(-3, 4, size=n, dtype=np.int64)
    a = rng.uniform(0.1, 1.0, size=n)
    bb = rng.standard_normal(n)
    cc = rng.standard_normal(n)
    coef = np.zeros((n, 5))
    coef[:, 4] = a
    coef[:, 3] = bb
    coef[:, 2] = cc
    return Instance(name=f"quartic_m{m}_n{n}_s{seed}", A=A, b=A @ x0,
                    l=np.full(n, -20, np.int64), u=np.full(n, 20, np.int64),
                    x0=x0, f_kind="separable_poly", coef=coef,
                    meta=dict(law="quartic", seed=seed))


def sparse_quadratic_instance(seed: int, n: int, m: int) -> Instance:
    """Batch-mix instance: A entries 0 w.p. 0.8 else uniform in {+-1, +-2};
    x0 uniform integers in [-2, 2]; l = -5, u = 5; quadratic f with
    Q = M^T M (M n x n iid uniform in [-2, 2]) and c iid uniform in [-5, 5]."""
    rng = _rng(seed)
    while True:
        nz = rng.random((m, n)) < 0.2
        mag = rng.integers(1, 3, size=(m, n))
        sg = np.where(rng.random((m, n)) < 0.5, -1, 1)
        A = (nz * mag * sg).astype(np.int64)
        if _full_row_rank(A):
            break
    x0 = rng.integers(-2, 3, size=n, dtype=np.int64)
    M = rng.integers(-2, 3, size=(n, n), dtype=np.int64)
    Q = (M.T @ M).astype(np.float64)
    c = rng.integers(-5, 6, size=n, dtype=np.int64).astype(np.float64)
    return Instance(name=f"mix_m{m}_n{n}_s{seed}", A=A, b=A @ x0,
                    l=np.full(n, -5, np.int64), u=np.full(n, 5, np.int64),
                    x0=x0, f_kind="quadratic", Q=Q, c=c,
                    meta=dict(law="mix", seed=seed))


def identity_block_instance(seed: int, n: int, m: int, density: float = 0.2) -> Instance:
    """Large-shape instance with an identity block: A = [I_m | C], C with
    entries 0 w.p. 1 - density else uniform in {+-1, +-2}; x0 uniform
    integers in [-2, 2]; l = -5, u = 5; quadratic f with Q = M^T M
    (M iid uniform in [-2, 2]) and c iid uniform in [-5, 5].  The identity
    block keeps the integer kernel basis computation cheap at large n."""
    rng = _rng(seed)
    d = n - m
    nz = rng.random((m, d)) < density
    mag = rng.integers(1, 3, size=(m, d))
    sg = np.where(rng.random((m, d)) < 0.5, -1, 1)
    C = (nz * mag * sg).astype(np.int64)
    A = np.concatenate([np.eye(m, dtype=np.int64), C], axis=1)
    x0 = rng.integers(-2, 3, size=n, dtype=np.int64)
    M = rng.integers(-2, 3, size=(n, n), dtype=np.int64)
    Q = (M.T @ M).astype(np.float64)
    c = rng.integers(-5, 6, size=n, dtype=np.int64).astype(np.float64)
    return Instance(name=f"idblock_m{m}_n{n}_s{seed}", A=A, b=A @ x0,
                    l=np.full(n, -5, np.int64), u=np.full(n, 5, np.int64),
                    x0=x0, f_kind="quadratic", Q=Q, c=c,
                    meta=dict(law="identity_block", seed=seed))


def inequality_rows(inst: Instance, mi: int, seed: int, nnz: int = 4, mag: int = 1):
    """Inequalities G x >= h that the instance's x0 satisfies: each row of G
    has `nnz` distinct random columns with entries uniform in
    {+-1, ..., +-mag}; h = G x0 - t with t uniform in {0, ..., 3}.
    Returns (G (mi, n) int64, h (mi,) int64)."""
    rng = _rng(seed)
    n = inst.n
    G = np.zeros((mi, n), np.int64)
    for i in range(mi):
        cols = rng.choice(n, size=nnz, replace=False)
        vals = rng.integers(1, mag + 1, size=nnz) * np.where(rng.random(nnz) < 0.5, -1, 1)
        G[i, cols] = vals
    h = G @ inst.x0 - rng.integers(0, 4, size=mi)
    return G, h.astype(np.int64)


def random_instance(seed: int, m: int, n: int, lo: int = -3, hi: int = 3,
                    bound: int = 5, density: float = 1.0) -> Instance:
    """Small random instance for tests: A iid uniform integers in [lo, hi]
    with the given density (redrawn until full row rank), x0 uniform in
    [-2, 2], box [-bound, bound], quadratic f with Q = M^T M (M iid in
    [-2, 2]) and c iid uniform integers in [-5, 5]."""
    rng = _rng(seed)
    while True:
        A = rng.integers(lo, hi + 1, size=(m, n), dtype=np.int64)
        if density < 1.0:
            A = A * (rng.random((m, n)) < density)
        if _full_row_rank(A):
            break
    x0 = rng.integers(-2, 3, size=n, dtype=np.int64)
    M = rng.integers(-2, 3, size=(n, n), dtype=np.int64)
    Q = (M.T @ M).astype(np.float64)
    c = rng.integers(-5, 6, size=n, dtype=np.int64).astype(np.float64)
    return Instance(name=f"rand_m{m}_n{n}_s{seed}", A=A, b=A @ x0,
                    l=np.full(n, -bound, np.int64), u=np.full(n, bound, np.int64),
                    x0=x0, f_kind="quadratic", Q=Q, c=c,
                    meta=dict(law="random", seed=seed))


def gaussian_starts(n_starts: int, d: int, sigma: float, seed: int) -> np.ndarray:
    """Start coordinates z0 ~ N(0, sigma^2 I), shape (n_starts, d), float64."""
    return _rng(seed).standard_normal((n_starts, d)) * sigma


def box_points(n_starts: int, l: np.ndarray, u: np.ndarray, seed: int) -> np.ndarray:
    """Points g ~ Uniform(l - u, u - l) componentwise, shape (n_starts, n)."""
    lo = (l - u).astype(np.float64)
    hi = (u - l).astype(np.float64)
    return lo + _rng(seed).random((n_starts, l.shape[0])) * (hi - lo)


def feasible_walk_starts(x0: np.ndarray, dirs: np.ndarray, l: np.ndarray,
                         u: np.ndarray, n_starts: int, seed: int,
                         walk_len: int = 64) -> np.ndarray:
    """Feasible augmentation starts: x0 followed by points of a seeded random
    walk x <- x +- g over the rows of ``dirs`` (integer kernel vectors), each
    move kept only when it stays inside [l, u].  Every returned row satisfies
    A x = b when x0 does.  Shape (n_starts, n), int64."""
    rng = _rng(seed)
    out = np.empty((n_starts, x0.shape[0]), np.int64)
    out[0] = x0
    x = x0.copy()
    for s in range(1, n_starts):
        if dirs.shape[0] > 0:
            for _ in range(walk_len):
                g = dirs[rng.integers(0, dirs.shape[0])].astype(np.int64)
                y = x + g if rng.random() < 0.5 else x - g
                if np.all(y >= l) and np.all(y <= u):
                    x = y
        out[s] = x
    return out


def combination_directions(B: np.ndarray, count: int, density: float, limit: int,
                           seed: int) -> np.ndarray:
    """A synthetic direction set of integer kernel vectors: ``count`` sparse
    integer combinations g = B z (z_j in {-1, 0, 1}, nonzero with probability
    ``density``), kept when 0 < |g_i| <= limit for every i, made unique, each
    with its first nonzero entry positive, in lexicographic order.  int64,
    shape (K, n)."""
    rng = _rng(seed)
    d = B.shape[1]
    Z = rng.integers(-1, 2, size=(count, d)) * (rng.random((count, d)) < density)
    G = Z @ np.asarray(B, dtype=np.int64).T
    G = G[np.all(np.abs(G) <= limit, axis=1) & np.any(G != 0, axis=1)]
    first = G[np.arange(G.shape[0]), np.argmax(G != 0, axis=1)]
    G = G * np.where(first < 0, -1, 1)[:, None]
    return np.unique(G, axis=0)


def antichain_with_sums(n: int, n_atoms: int, support: int, n_sums: int, seed: int,
                        mag: int = 3, positive: bool = False) -> tuple:
    """Key set whose minimal elements are known in closed form.

    Atoms: n_atoms int8 rows with exactly `support` nonzeros (values in
    +-1..+-mag) on pairwise distinct supports; rows with distinct supports
    of one size never lie conformally below one another, or below each
    other's negation.  positive=True makes every atom nonnegative (all
    keys then share few sign patterns).  Sums: a + b for random atom pairs whose signs agree
    wherever both are nonzero (a lies conformally below a + b).  The rows
    are shuffled, about half are negated, and some sums are repeated.
    Returns (X, atoms): X the int8 key set, atoms its minimal elements.
    """
    rng = _rng(seed)
    sup = set()
    rows = []
    while len(rows) < n_atoms:
        s = tuple(sorted(rng.choice(n, size=support, replace=False).tolist()))
        if s in sup:
            continue
        sup.add(s)
        r = np.zeros(n, np.int64)
        sgn = 1 if positive else rng.choice([-1, 1], size=support)
        r[list(s)] = rng.integers(1, mag + 1, size=support) * sgn
        rows.append(r)
    atoms = np.array(rows, dtype=np.int64)
    sums = []
    while len(sums) < n_sums:
        i = rng.integers(0, n_atoms, size=2 * n_sums)
        j = rng.integers(0, n_atoms, size=2 * n_sums)
        ok = (i != j) & np.all(atoms[i] * atoms[j] >= 0, axis=1)
        s = atoms[i[ok]] + atoms[j[ok]]
        sums.extend(s[: n_sums - len(sums)])
    S = np.array(sums, dtype=np.int64)
    X = np.concatenate([atoms, S, S[: n_sums // 10]])
    X = X[rng.permutation(X.shape[0])]
    X[rng.random(X.shape[0]) < 0.5] *= -1
    return X.astype(np.int8), atoms

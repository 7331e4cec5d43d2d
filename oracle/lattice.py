"""Integer kernel basis of A (Section 3.1) -- oracle, test infrastructure only.

* ``hnf_kernel_basis`` -- Lemma 3.1: a unimodular K with A K = (H | 0), H in
  Hermite normal form; B is the last d = n - rank(A) columns of K and spans
  Ker_Z(A) (Theorem 3.2).
* ``lll_reduce`` -- Appendix A, Algorithm 3 (LLL with the size condition
  |mu_ij| <= 1/2 and the exchange condition ||B*_j||^2 <= 2 ||B*_{j+1}||^2).
* ``coordinate_projector`` -- the inverse map z = (B^T B)^-1 B^T g of
  Section 3.1.

All integer work uses Python ints (no overflow).  The column operations of
the HNF are fixed (smallest nonzero pivot, ties to the lowest column, floor
quotients), so K and B are a deterministic function of A.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List

import numpy as np


def _round_half_even(q: Fraction) -> int:
    """Nearest integer to a rational, ties to even (the paper's nearest-integer
    bracket; ties are not specified there)."""
    return round(q)  # Fraction.__round__ rounds half to even


def hnf_kernel_basis(A) -> dict:
    """Column-style Hermite normal form by unimodular column operations.

    Rows are processed in order.  In row i, among the not-yet-pivoted
    columns p..n-1, the nonzero entry of smallest absolute value (ties to the
    lowest column index) is moved to column p and every other column k > p
    is reduced by floor(a_ik / a_ip) times column p; this repeats until
    column p is the only nonzero entry of row i among p..n-1.  The pivot is
    made positive, the entries of row i left of the pivot are reduced into
    [0, pivot), and p advances.  A row with no nonzero entry in p..n-1 is
    linearly dependent on earlier rows and yields no pivot.

    Returns dict(K=n x n, H=m x rank, rank=r, B=n x (n-r)) as lists of ints.
    """
    A = [[int(v) for v in row] for row in np.asarray(A).tolist()]
    m = len(A)
    n = len(A[0]) if m else 0
    W = [row[:] for row in A]  # W = A K, kept in sync with K
    K = [[1 if i == j else 0 for j in range(n)] for i in range(n)]

    def col_axpy(dst, src, q):  # column dst -= q * column src
        for row in W:
            row[dst] -= q * row[src]
        for row in K:
            row[dst] -= q * row[src]

    def col_swap(a, b):
        for row in W:
            row[a], row[b] = row[b], row[a]
        for row in K:
            row[a], row[b] = row[b], row[a]

    def col_negate(a):
        for row in W:
            row[a] = -row[a]
        for row in K:
            row[a] = -row[a]

    p = 0
    for i in range(m):
        if p == n:
            break
        pivoted = False
        while True:
            nz = [k for k in range(p, n) if W[i][k] != 0]
            if not nz:
                break
            piv = min(nz, key=lambda k: (abs(W[i][k]), k))
            if piv != p:
                col_swap(p, piv)
            pivoted = True
            clean = True
            for k in range(p + 1, n):
                if W[i][k] != 0:
                    q = W[i][k] // W[i][p]
                    col_axpy(k, p, q)
                    if W[i][k] != 0:
                        clean = False
            if clean:
                break
        if not pivoted:
            continue
        if W[i][p] < 0:
            col_negate(p)
        for j in range(p):
            q = W[i][j] // W[i][p]
            if q != 0:
                col_axpy(j, p, q)
        p += 1
    r = p
    B = [row[r:] for row in K]
    H = [row[:r] for row in W]
    return dict(K=K, H=H, rank=r, B=B)


def gram_schmidt_exact(cols: List[List[int]]):
    """Exact rational Gram-Schmidt of the basis vectors ``cols`` (each a list
    of ints): returns (mu, bstar_norm2) with mu[i][j] = <b_i, b*_j>/<b*_j, b*_j>
    for j < i (Appendix A).  Used by tests to check the reduced-basis
    conditions; the reduction itself works in integers."""
    d = len(cols)
    bstar: List[List[Fraction]] = []
    norm2: List[Fraction] = []
    mu = [[Fraction(0)] * d for _ in range(d)]
    for i in range(d):
        v = [Fraction(x) for x in cols[i]]
        for j in range(i):
            num = sum(Fraction(a) * b for a, b in zip(cols[i], bstar[j]))
            mu[i][j] = num / norm2[j]
            v = [vi - mu[i][j] * bj for vi, bj in zip(v, bstar[j])]
        bstar.append(v)
        norm2.append(sum(x * x for x in v))
    return mu, norm2


def lll_reduce(B, factor: int = 2) -> List[List[int]]:
    """LLL reduction of the columns of B (n x d), Appendix A, Algorithm 3.

    The paper's order of steps: with i starting at the second vector, size
    reduce b_i against b_{i-1}, ..., b_1 (b_i <- b_i - [mu_ij] b_j, nearest
    integer with ties to even), then exchange b_i and b_{i-1} when
    ||b*_{i-1}||^2 > factor * ||b*_i||^2 and step back (never below the
    second vector), otherwise advance.  It stops when i passes the last
    vector.

    The Gram-Schmidt data are carried exactly in the integral form of the
    same quantities (Cohen, "A Course in Computational Algebraic Number
    Theory", Sec. 2.6): D[k] = prod_{j<k} ||b*_j||^2 (Gram determinants,
    D[0] = 1) and lam[i][j] = D[j+1] * mu_ij, so every test and every
    rounding is decided on exact integers:
        mu_ij = lam[i][j] / D[j+1],   ||b*_k||^2 = D[k+1] / D[k].
    """
    Bm = [[int(v) for v in row] for row in B]
    n = len(Bm)
    d = len(Bm[0]) if n else 0
    b = [[Bm[r][c] for r in range(n)] for c in range(d)]  # columns as vectors

    def dot(x, y):
        return sum(p * q for p, q in zip(x, y))

    # Integral Gram-Schmidt.
    D = [1] + [0] * d
    lam = [[0] * d for _ in range(d)]
    for k in range(d):
        for j in range(k + 1):
            u = dot(b[k], b[j])
            for i in range(j):
                u = (D[i + 1] * u - lam[k][i] * lam[j][i]) // D[i]
            if j < k:
                lam[k][j] = u
            else:
                if u == 0:
                    raise ValueError("basis vectors are linearly dependent")
                D[k + 1] = u

    def size_reduce(k, j):
        q = _round_half_even(Fraction(lam[k][j], D[j + 1]))
        if q != 0:
            b[k] = [x - q * y for x, y in zip(b[k], b[j])]
            lam[k][j] -= q * D[j + 1]
            for i in range(j):
                lam[k][i] -= q * lam[j][i]

    def exchange(k):  # swap b_k and b_{k-1} (0-indexed k >= 1)
        b[k], b[k - 1] = b[k - 1], b[k]
        for j in range(k - 1):
            lam[k][j], lam[k - 1][j] = lam[k - 1][j], lam[k][j]
        lk = lam[k][k - 1]
        Bnew = (D[k - 1] * D[k + 1] + lk * lk) // D[k]
        for i in range(k + 1, d):
            t = lam[i][k]
            lam[i][k] = (D[k + 1] * lam[i][k - 1] - lk * t) // D[k]
            lam[i][k - 1] = (Bnew * t + lk * lam[i][k]) // D[k + 1]
        D[k] = Bnew

    i = 1
    while i < d:
        for j in range(i - 1, -1, -1):
            size_reduce(i, j)
        # ||b*_{i-1}||^2 > factor ||b*_i||^2  <=>  D[i]^2 > factor D[i+1] D[i-1]
        if D[i] * D[i] > factor * D[i + 1] * D[i - 1]:
            exchange(i)
            i = max(i - 1, 1)
        else:
            i += 1
    return [[b[c][r] for c in range(d)] for r in range(n)]


def kernel_basis(A, lll: bool = True) -> np.ndarray:
    """B (n x d int64): HNF kernel columns, LLL-reduced when ``lll``."""
    B = hnf_kernel_basis(A)["B"]
    if lll and B and B[0]:
        B = lll_reduce(B)
    return np.array(B, dtype=np.int64).reshape(len(B), -1)


def coordinate_projector(B) -> np.ndarray:
    """P = (B^T B)^-1 B^T (d x n, float64), Section 3.1.

    Computed exactly in rationals and rounded once to binary64 per entry, so
    it is a fixed function of B."""
    Bl = [[int(v) for v in row] for row in np.asarray(B).tolist()]
    n = len(Bl)
    d = len(Bl[0])
    G = [[Fraction(sum(Bl[r][i] * Bl[r][j] for r in range(n))) for j in range(d)]
         for i in range(d)]
    # Gauss-Jordan inverse of the Gram matrix in exact rationals.
    M = [G[i][:] + [Fraction(int(i == j)) for j in range(d)] for i in range(d)]
    for col in range(d):
        piv = next(r for r in range(col, d) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [x / pv for x in M[col]]
        for r in range(d):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    Ginv = [row[d:] for row in M]
    P = np.empty((d, n))
    for i in range(d):
        for r in range(n):
            P[i, r] = float(sum(Ginv[i][j] * Bl[r][j] for j in range(d)))
    return P

"""Conformal order, Graver basis by brute force, kernel check -- oracle, test
infrastructure only.

Section 1 defines x <= y (conformal order) as x_i y_i >= 0 and |x_i| <= |y_i|
for every i, and the Graver basis G(A) as the conformally minimal elements of
Ker_Z(A) \\ {0}.  Condition C1 of Section 3 is A g = 0.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np


def conformal_le(h: Sequence[int], g: Sequence[int]) -> bool:
    """h conformally below g: h_i g_i >= 0 and |h_i| <= |g_i| for all i."""
    return all(a * b >= 0 and abs(a) <= abs(b) for a, b in zip(h, g))


def in_kernel(A, g: Sequence[int]) -> bool:
    """Condition C1: A g = 0, in exact integers."""
    A = np.asarray(A)
    return all(sum(int(A[i, j]) * int(g[j]) for j in range(len(g))) == 0
               for i in range(A.shape[0]))


def canonical(g: Sequence[int]) -> Tuple[int, ...]:
    """Representative of {g, -g}: the one whose first nonzero entry is > 0."""
    for x in g:
        if x != 0:
            return tuple(int(v) for v in g) if x > 0 else tuple(-int(v) for v in g)
    return tuple(int(v) for v in g)


def _rref_pivots(A) -> List[int]:
    """Pivot columns of the reduced row echelon form of A (exact rationals)."""
    M = [[Fraction(int(v)) for v in row] for row in np.asarray(A).tolist()]
    m = len(M)
    n = len(M[0]) if m else 0
    piv = []
    r = 0
    for c in range(n):
        p = next((i for i in range(r, m) if M[i][c] != 0), None)
        if p is None:
            continue
        M[r], M[p] = M[p], M[r]
        pv = M[r][c]
        M[r] = [x / pv for x in M[r]]
        for i in range(m):
            if i != r and M[i][c] != 0:
                f = M[i][c]
                M[i] = [x - f * y for x, y in zip(M[i], M[r])]
        piv.append(c)
        r += 1
        if r == m:
            break
    return piv


def _det_adj(M: List[List[Fraction]]):
    """Determinant and adjugate of a small square rational matrix."""
    r = len(M)
    if r == 0:
        return Fraction(1), []
    # inverse by Gauss-Jordan, then adj = det * inv
    aug = [row[:] + [Fraction(int(i == j)) for j in range(r)] for i, row in enumerate(M)]
    det = Fraction(1)
    for c in range(r):
        p = next(i for i in range(c, r) if aug[i][c] != 0)
        if p != c:
            aug[c], aug[p] = aug[p], aug[c]
            det = -det
        pv = aug[c][c]
        det *= pv
        aug[c] = [x / pv for x in aug[c]]
        for i in range(r):
            if i != c and aug[i][c] != 0:
                f = aug[i][c]
                aug[i] = [x - f * y for x, y in zip(aug[i], aug[c])]
    inv = [row[r:] for row in aug]
    adj = [[det * x for x in row] for row in inv]
    return det, adj


def kernel_vectors_in_box(A, R: int) -> np.ndarray:
    """All nonzero g in Z^n with A g = 0 and |g_i| <= R, by enumeration.

    The free (non-pivot) coordinates run over [-R, R]^(n-r); the pivot
    coordinates are then fixed by A g = 0 and kept only when integral and
    inside the box.  Returns an (K, n) int64 array."""
    A = np.asarray(A, dtype=np.int64)
    m, n = A.shape
    piv = _rref_pivots(A)
    r = len(piv)
    rows = _rref_rows(A, piv)
    free = [c for c in range(n) if c not in piv]
    Ap = [[Fraction(int(A[i, c])) for c in piv] for i in rows]
    det, adj = _det_adj(Ap)
    det_i = int(det)
    adj_i = np.array([[int(x) for x in row] for row in adj], dtype=np.int64).reshape(r, r)
    Af = A[np.ix_(rows, free)]
    # x_piv * det = -adj @ Af @ x_free
    T = -(adj_i @ Af)  # (r, n-r) integer
    k = len(free)
    vals = np.arange(-R, R + 1, dtype=np.int64)
    out = []
    total = (2 * R + 1) ** k
    chunk = 1 << 18
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        xf = np.empty((idx.size, k), np.int64)
        rem = idx.copy()
        for j in range(k - 1, -1, -1):
            xf[:, j] = vals[rem % (2 * R + 1)]
            rem //= (2 * R + 1)
        num = xf @ T.T  # (chunk, r) = det * x_piv
        ok = np.all(num % det_i == 0, axis=1)
        xp = num // det_i
        ok &= np.all(np.abs(xp) <= R, axis=1)
        g = np.zeros((idx.size, n), np.int64)
        g[:, free] = xf
        g[:, piv] = xp
        ok &= np.any(g != 0, axis=1)
        out.append(g[ok])
    G = np.concatenate(out) if out else np.zeros((0, n), np.int64)
    assert np.all(G @ A.T == 0)
    return G


def _rref_rows(A, piv: List[int]) -> List[int]:
    """Indices of r linearly independent rows of A whose restriction to the
    pivot columns is invertible."""
    A = np.asarray(A)
    chosen: List[int] = []
    for i in range(A.shape[0]):
        trial = chosen + [i]
        M = [[Fraction(int(A[a, c])) for c in piv] for a in trial]
        if _rank(M) == len(trial):
            chosen = trial
        if len(chosen) == len(piv):
            break
    return chosen


def _rank(M: List[List[Fraction]]) -> int:
    M = [row[:] for row in M]
    rank = 0
    cols = len(M[0]) if M else 0
    for c in range(cols):
        p = next((i for i in range(rank, len(M)) if M[i][c] != 0), None)
        if p is None:
            continue
        M[rank], M[p] = M[p], M[rank]
        for i in range(len(M)):
            if i != rank and M[i][c] != 0:
                f = M[i][c] / M[rank][c]
                M[i] = [x - f * y for x, y in zip(M[i], M[rank])]
        rank += 1
    return rank


def minimal_elements(V: np.ndarray) -> np.ndarray:
    """Conformally minimal rows of V (rows nonzero).

    Rows are taken level by level in increasing l1 norm; since h <= g with
    h != g forces ||h||_1 < ||g||_1, a row is minimal iff no minimal row of a
    lower level lies conformally below it."""
    V = np.asarray(V, dtype=np.int64)
    if V.shape[0] == 0:
        return V
    l1 = np.abs(V).sum(axis=1)
    keep_rows = []
    Gmin = np.zeros((0, V.shape[1]), np.int64)
    for level in np.unique(l1):
        L = V[l1 == level]
        if Gmin.shape[0] == 0:
            survivors = L
        else:
            dead = np.zeros(L.shape[0], bool)
            for s in range(0, L.shape[0], 512):
                blk = L[s:s + 512]
                # h <= g  <=>  h*g >= 0 and |h| <= |g| componentwise
                prod_ok = (Gmin[None, :, :] * blk[:, None, :]) >= 0
                mag_ok = np.abs(Gmin)[None, :, :] <= np.abs(blk)[:, None, :]
                dead[s:s + 512] = np.any(np.all(prod_ok & mag_ok, axis=2), axis=1)
            survivors = L[~dead]
        keep_rows.append(survivors)
        Gmin = np.concatenate([Gmin, survivors])
    return Gmin


def graver_basis_in_box(A, R: int) -> List[Tuple[int, ...]]:
    """G(A) intersected with the box [-R, R]^n, by brute force: every nonzero
    kernel vector in the box, minus those with a conformally smaller kernel
    vector.  Exact for the box because every h <= g lies in g's box.
    Returned as sorted tuples (both signs present)."""
    V = kernel_vectors_in_box(A, R)
    M = minimal_elements(V)
    return sorted(tuple(int(x) for x in row) for row in M)

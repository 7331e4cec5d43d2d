"""Pins for the oracle's kernel basis (Lemma 3.1, Theorem 3.2), LLL
(Appendix A) and coordinate map (Section 3.1)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import lattice
from oracle.conformal import kernel_vectors_in_box
from paper_2412_13576_amd import workloads as W


def _det(M):
    """Exact determinant (Bareiss fraction-free elimination)."""
    M = [[int(v) for v in row] for row in M]
    n = len(M)
    sign, prev = 1, 1
    for k in range(n - 1):
        if M[k][k] == 0:
            sw = next((i for i in range(k + 1, n) if M[i][k] != 0), None)
            if sw is None:
                return 0
            M[k], M[sw] = M[sw], M[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                M[i][j] = (M[i][j] * M[k][k] - M[i][k] * M[k][j]) // prev
        prev = M[k][k]
    return sign * M[n - 1][n - 1]


def _solve_exact(B, g):
    """z with B z = g for full-column-rank integer B, exactly, or None."""
    Bl = [[Fraction(int(v)) for v in row] for row in B]
    n, d = len(Bl), len(Bl[0])
    G = [[sum(Bl[r][i] * Bl[r][j] for r in range(n)) for j in range(d)] for i in range(d)]
    h = [sum(Bl[r][i] * int(g[r]) for r in range(n)) for i in range(d)]
    M = [G[i] + [h[i]] for i in range(d)]
    for c in range(d):
        p = next(r for r in range(c, d) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        M[c] = [x / M[c][c] for x in M[c]]
        for r in range(d):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    z = [M[i][d] for i in range(d)]
    if any(sum(Bl[r][j] * z[j] for j in range(d)) != int(g[r]) for r in range(n)):
        return None
    return z


CASES = [W.random_instance(s, m, n).A for s, (m, n) in enumerate([(1, 3), (2, 5), (2, 8), (3, 7), (4, 9)])]
CASES.append(np.array([[1, 2, 3, 4], [2, 4, 6, 8]], dtype=np.int64))      # rank deficient
CASES.append(np.array([[0, 0, 0], [1, -1, 2]], dtype=np.int64))            # zero row
CASES.append(np.array([[6, 10, 15]], dtype=np.int64))                      # gcd structure


@pytest.mark.parametrize("A", CASES)
def test_hnf_invariants(A):
    h = lattice.hnf_kernel_basis(A)
    K = np.array(h["K"], dtype=object)
    r = h["rank"]
    assert r == np.linalg.matrix_rank(A.astype(float))
    assert abs(_det(h["K"])) == 1                      # unimodular (Lemma 3.1)
    AK = A.astype(object) @ K
    assert np.all(AK[:, r:] == 0)                      # A B = 0
    H = AK[:, :r]
    # Hermite shape: each pivot positive, entries right of it zero, entries
    # left of it reduced into [0, pivot).
    prow = -1
    for c in range(r):
        rows = [i for i in range(A.shape[0]) if H[i, c] != 0]
        top = min(rows)
        assert top > prow and H[top, c] > 0
        for j in range(c):
            assert 0 <= H[top, j] < H[top, c]
        prow = top
    assert len(h["B"][0]) == A.shape[1] - r


@pytest.mark.parametrize("A", CASES[:6])
def test_theorem_3_2_every_kernel_vector_has_integral_coordinates(A):
    B = lattice.hnf_kernel_basis(A)["B"]
    for g in kernel_vectors_in_box(A, 2)[:400]:
        z = _solve_exact(B, g)
        assert z is not None and all(x.denominator == 1 for x in z)


def test_coprime_pair_closed_form():
    for a, b in [(3, 5), (2, 7), (-4, 9), (1, 1)]:
        B = np.array(lattice.hnf_kernel_basis(np.array([[a, b]]))["B"]).ravel()
        assert tuple(B) in {(b, -a), (-b, a)}


def _reduced(B, factor=2):
    cols = [[int(B[r][c]) for r in range(len(B))] for c in range(len(B[0]))]
    mu, nb = lattice.gram_schmidt_exact(cols)
    d = len(cols)
    cond_i = all(abs(mu[i][j]) <= Fraction(1, 2) for i in range(d) for j in range(i))
    cond_ii = all(nb[j] <= factor * nb[j + 1] for j in range(d - 1))
    return cond_i, cond_ii


@pytest.mark.parametrize("A", CASES[:5] + [W.tiny_instance(1000).A])
def test_lll_reduced_and_same_lattice(A):
    B0 = lattice.hnf_kernel_basis(A)["B"]
    B1 = lattice.lll_reduce(B0)
    c1, c2 = _reduced(B1)
    assert c1 and c2                                   # Appendix A (i), (ii)
    assert np.all(A.astype(object) @ np.array(B1, dtype=object) == 0)
    # same lattice: B1 = B0 U with U integral and |det U| = 1
    d = len(B0[0])
    U = [[None] * d for _ in range(d)]
    for c in range(d):
        z = _solve_exact(B0, [B1[r][c] for r in range(len(B1))])
        assert z is not None and all(x.denominator == 1 for x in z)
        for rr in range(d):
            U[rr][c] = int(z[rr])
    assert abs(_det(U)) == 1


def test_lll_reduces_a_skewed_basis():
    # A lattice basis with a long, nearly parallel second vector.
    B = [[1, 101], [0, 1], [1, 100]]
    R = lattice.lll_reduce(B)
    c1, c2 = _reduced(R)
    assert c1 and c2
    assert max(sum(R[r][c] ** 2 for r in range(3)) for c in range(2)) <= 3


def test_projector_inverts_basis():
    inst = W.tiny_instance(1000)
    B = lattice.kernel_basis(inst.A)
    P = lattice.coordinate_projector(B)
    assert np.abs(P @ B - np.eye(B.shape[1])).max() < 1e-14
    z = np.array([2, -1, 0, 3, 1, -2], dtype=float)[: B.shape[1]]
    assert np.allclose(P @ (B @ z), z, atol=1e-12)

"""Host-side checks of the C-ABI library (no GPU compute): it loads,
exports every declared entry point, and its host kernel basis matches the
oracle bit for bit."""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from oracle import lattice
from paper_2412_13576_amd import graver as G
from paper_2412_13576_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "graver.h")).read()
    return sorted(set(re.findall(r"\b(graver_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = G.lib()
    names = _declared()
    assert set(G.EXPORTED) == set(names)
    for name in names:
        assert hasattr(L, name), name


INSTANCES = [W.tiny_instance(s) for s in range(1000, 1005)] + [
    W.random_instance(7, 3, 9), W.random_instance(8, 4, 12, density=0.5), W.qp_instance(2000)]


@pytest.mark.parametrize("inst", INSTANCES, ids=[i.name for i in INSTANCES])
@pytest.mark.parametrize("lll", [False, True])
def test_host_kernel_basis_matches_oracle(inst, lll):
    B, P = G.kernel_basis(inst.A, lll=lll)
    Bo = lattice.kernel_basis(inst.A, lll=lll)
    assert np.array_equal(B, Bo)
    assert np.all(inst.A @ B == 0)
    if lll and inst.n <= 12:
        Po = lattice.coordinate_projector(Bo)
        assert np.allclose(P, Po, rtol=1e-13, atol=1e-15)


def test_host_kernel_basis_rank_deficient_and_errors():
    A = np.array([[1, 2, 3, 4], [2, 4, 6, 8]])
    B, P = G.kernel_basis(A)
    assert B.shape == (4, 3) and np.array_equal(B, lattice.kernel_basis(A))
    with pytest.raises(G.GraverError) as e:
        G.lib()  # loaded
        import ctypes as C
        d = C.c_int32(0)
        G._check(G.lib().graver_kernel_basis(0, 4, None, 1, None, C.byref(d), None))
    assert e.value.status == -1


def test_host_kernel_basis_overflow_is_reported():
    # The exact K of this A has entries of 150+ bits, which int64 cannot hold.
    A = np.array([[2 ** 40 + 1, 2 ** 40 + 3, 5], [7, 11, 2 ** 40 + 13]], dtype=np.int64)
    h = lattice.hnf_kernel_basis(A)
    assert max(abs(v) for row in h["K"] for v in row) >= 2 ** 63
    with pytest.raises(G.GraverError) as e:
        G.kernel_basis(A, lll=False)
    assert e.value.status == -4
    # large but representable entries still match the oracle exactly
    A = np.array([[2 ** 50 + 1, 2 ** 50 + 3, 2 ** 49 + 5]], dtype=np.int64)
    B, _ = G.kernel_basis(A, lll=False)
    assert np.array_equal(B, np.array(lattice.hnf_kernel_basis(A)["B"], dtype=np.int64))


def test_lift_inequalities_matches_oracle():
    """The host slack form and lifted basis equal the oracle's, bit for bit."""
    from oracle import inequality as Q
    for inst, mi, seed in [(W.tiny_instance(1000), 2, 1), (W.qp_instance(2000), 10, 2), (W.quartic_instance(), 6, 3)]:
        Gm, h = W.inequality_rows(inst, mi, seed, nnz=4, mag=2)
        B = lattice.kernel_basis(inst.A) if inst.n <= 100 else None
        A2, b2, l2, u2, Bt = G.lift_inequalities(inst.A, inst.b, inst.l, inst.u, Gm, h, B)
        Ao, bo, lo, uo = Q.lift(inst.A, inst.b, inst.l, inst.u, Gm, h)
        assert np.array_equal(A2, Ao) and np.array_equal(b2, bo)
        assert np.array_equal(l2, lo) and np.array_equal(u2, uo)
        if B is not None:
            assert np.array_equal(Bt, Q.lift_basis(B, Gm))
            assert np.all(A2 @ Bt == 0)
        assert np.all(A2 @ Q.lift_point(inst.x0, Gm, h) == b2)


def test_lift_inequalities_errors():
    inst = W.tiny_instance(1000)
    Gm = np.ones((1, 8), np.int64)
    with pytest.raises(G.GraverError) as e:
        G.lift_inequalities(inst.A, inst.b, inst.l, inst.u, Gm, np.array([100]))
    assert e.value.status == G.GRAVER_E_INVALID
    with pytest.raises(G.GraverError) as e:
        G.lift_inequalities(inst.A, inst.b, inst.l, inst.u, Gm * (1 << 60), np.array([0]))
    assert e.value.status == G.GRAVER_E_OVERFLOW


def _hermite_is_identity(B):
    """The rows of B (n x d) generate Z^d, i.e. B is primitive: the oracle's
    Hermite form of the lattice spanned by the rows is the identity."""
    H = lattice.hnf_kernel_basis(B.T)["H"]
    d = B.shape[1]
    return len(H) == d and all(int(H[i][j]) == (1 if i == j else 0) for i in range(d) for j in range(d))


@pytest.mark.parametrize("n,m", [(150, 45), (300, 60)])
def test_iid_sparse_law_basis_spans_the_kernel_lattice(n, m):
    """The batching law (A iid, 0 w.p. 0.8 else +-1, +-2): the kernel columns
    of the Hermite normal form of Lemma 3.1 leave int64 (the oracle's, in
    exact integers, do), so the library reduces while it eliminates.  Its
    basis must still span Ker_Z(A) (Theorem 3.2): A B = 0, d = n - rank(A),
    and B primitive, which with A B = 0 and full rank d makes L(B) the whole
    kernel lattice; its entries stay within the matrix-core descent's limits."""
    inst = W.sparse_quadratic_instance(4000 + n, n, m)
    ho = lattice.hnf_kernel_basis(inst.A)
    assert max(abs(int(x)) for r in ho["B"] for x in r) >= 2 ** 63
    B, P = G.kernel_basis(inst.A, lll=True)
    assert B.shape == (n, n - ho["rank"])
    assert not np.any(inst.A @ B)
    assert _hermite_is_identity(B)
    assert np.abs(B).max() <= 256 and np.abs(B).sum(axis=1).max() * 256 < 2 ** 24
    assert np.allclose(P @ B, np.eye(B.shape[1]), atol=1e-6)  # the start map z = P g


def test_iid_sparse_law_basis_is_reduced():
    """The reduced basis of that path satisfies Appendix A's exchange
    condition (ii) ||b*_j||^2 <= 2 ||b*_{j+1}||^2 exactly and the size
    condition (i) up to the reduction's bound |mu_ij| <= 0.51 (checked with
    the oracle's exact rational Gram-Schmidt)."""
    inst = W.sparse_quadratic_instance(4150, 150, 45)
    B, _ = G.kernel_basis(inst.A, lll=True)
    cols = [[int(B[r][c]) for r in range(B.shape[0])] for c in range(B.shape[1])]
    mu, nb = lattice.gram_schmidt_exact(cols)
    d = len(cols)
    assert all(nb[j] <= 2 * nb[j + 1] for j in range(d - 1))
    assert all(abs(mu[i][j]) <= Fraction(51, 100) for i in range(d) for j in range(i))

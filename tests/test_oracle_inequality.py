"""Pins of the inequality lift (Section 3.4)."""
import itertools

import numpy as np

from oracle import conformal, inequality as Q, lattice
from paper_2412_13576_amd import workloads as W


def _case():
    inst = W.tiny_instance(1000)
    G = np.array([[1, 1, 0, 0, -1, 0, 0, 0], [0, 0, 1, -1, 0, 1, 0, 1]], dtype=np.int64)
    h = np.array([-3, -4], dtype=np.int64)
    return inst, G, h


def test_lifted_basis_spans_the_lifted_kernel():
    """Corollary: Ker_Z([A 0; G -I]) = L([B; GB]).  Both directions are
    checked against an independently computed kernel basis of the lifted
    matrix: each basis expresses the other's columns with integer
    coefficients (exact rational solves)."""
    from fractions import Fraction
    inst, G, h = _case()
    A2, _, _, _ = Q.lift(inst.A, inst.b, inst.l, inst.u, G, h)
    B = lattice.kernel_basis(inst.A)
    Bt = Q.lift_basis(B, G)
    assert np.all(A2 @ Bt == 0)
    K = lattice.kernel_basis(A2, lll=False)
    assert K.shape[1] == Bt.shape[1]

    def int_coords(M, v):
        # solve M c = v exactly (M has full column rank); return c or None
        Mf = [[Fraction(int(x)) for x in row] for row in M]
        rows, cols = len(Mf), len(Mf[0])
        aug = [Mf[r] + [Fraction(int(v[r]))] for r in range(rows)]
        piv = []
        r = 0
        for c in range(cols):
            p = next((i for i in range(r, rows) if aug[i][c] != 0), None)
            if p is None:
                continue
            aug[r], aug[p] = aug[p], aug[r]
            for i in range(rows):
                if i != r and aug[i][c] != 0:
                    f = aug[i][c] / aug[r][c]
                    aug[i] = [a - f * bb for a, bb in zip(aug[i], aug[r])]
            piv.append(c)
            r += 1
        assert all(all(x == 0 for x in aug[i][:cols]) <= (aug[i][cols] == 0) for i in range(r, rows))
        coef = [aug[i][cols] / aug[i][c] for i, c in enumerate(piv)]
        return coef

    for j in range(K.shape[1]):
        assert all(c.denominator == 1 for c in int_coords(Bt, K[:, j]))
    for j in range(Bt.shape[1]):
        assert all(c.denominator == 1 for c in int_coords(K, Bt[:, j]))


def test_lift_keeps_exactly_the_feasible_points():
    """x in the box satisfies A x = b and G x >= h iff (x, G x - h) is
    feasible for the lifted program (exhaustive over a small box)."""
    A = np.array([[1, 2, -1]], dtype=np.int64)
    b = np.array([1], dtype=np.int64)
    l = np.full(3, -2, np.int64)
    u = np.full(3, 2, np.int64)
    G = np.array([[1, -1, 1], [0, 2, 1]], dtype=np.int64)
    h = np.array([-1, 0], dtype=np.int64)
    A2, b2, l2, u2 = Q.lift(A, b, l, u, G, h)
    for x in itertools.product(range(-2, 3), repeat=3):
        x = np.array(x)
        ok = np.all(A @ x == b) and np.all(G @ x >= h)
        y = Q.lift_point(x, G, h)
        ok2 = np.all(A2 @ y == b2) and np.all((y >= l2) & (y <= u2))
        assert ok == ok2


def test_lifted_graver_basis_projects_to_sign_compatible_moves():
    """Every Graver element of the lifted matrix (enumerated in a box) is
    (g, G g) for an integer kernel vector g of A."""
    A = np.array([[1, 1, 1]], dtype=np.int64)
    G = np.array([[1, 0, -1]], dtype=np.int64)
    A2 = np.concatenate([np.concatenate([A, np.zeros((1, 1), np.int64)], 1),
                         np.concatenate([G, -np.eye(1, dtype=np.int64)], 1)])
    Gr = conformal.graver_basis_in_box(A2, 3)
    assert len(Gr) > 0
    for g in Gr:
        g = np.array(g)
        assert np.all(A @ g[:3] == 0) and g[3] == G[0] @ g[:3]


def test_slack_bounds_are_the_largest_slack_in_the_box():
    l = np.array([-2, 0, -1])
    u = np.array([3, 4, 1])
    G = np.array([[2, -1, 3], [-1, -1, 0]])
    h = np.array([1, -2])
    best = [max(int(G[i] @ np.array(x)) - h[i] for x in itertools.product(*[range(a, b + 1) for a, b in zip(l, u)]))
            for i in range(2)]
    assert list(Q.slack_bounds(G, h, l, u)) == best

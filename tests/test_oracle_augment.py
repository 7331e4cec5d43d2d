"""Pins for the augmentation scheme (Algorithm 1, Proposition 2.1) and the
objective evaluation."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle.augment import Augmenter, Objective, augment, objective
from oracle.conformal import graver_basis_in_box, canonical
from paper_2412_13576_amd import workloads as W


def _exact_f(f, x):
    if f.kind == "quadratic":
        n = len(x)
        return sum(Fraction(f.Q[i, j]) * x[i] * x[j] for i in range(n) for j in range(n)) + \
            sum(Fraction(f.c[i]) * x[i] for i in range(n))
    return sum(Fraction(f.coef[i, k]) * Fraction(int(x[i])) ** k
               for i in range(len(x)) for k in range(f.coef.shape[1]))


def _feasible_points(A, b, l, u):
    n = A.shape[1]
    pts = []
    for x in itertools.product(*[range(int(l[i]), int(u[i]) + 1) for i in range(n)]):
        if np.all(A @ np.array(x) == b):
            pts.append(np.array(x, dtype=np.int64))
    return pts


def _tiny():
    A = np.array([[1, 1, 1, 0, 2], [0, 1, -1, 1, 1]], dtype=np.int64)
    x0 = np.array([1, 0, -1, 2, 0], dtype=np.int64)
    l = np.full(5, -2, np.int64)
    u = np.full(5, 2, np.int64)
    return A, A @ x0, l, u, x0


def test_objective_exact_on_integer_data():
    inst = W.tiny_instance(1000)
    f = Objective("quadratic", Q=inst.Q, c=inst.c)
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.integers(-5, 6, size=8)
        assert objective(f, x) == float(_exact_f(f, x))
    coef = rng.integers(-3, 4, size=(8, 5)).astype(float)
    fp = Objective("separable_poly", coef=coef)
    for _ in range(20):
        x = rng.integers(-5, 6, size=8)
        assert objective(fp, x) == float(_exact_f(fp, x))


@pytest.mark.parametrize("kind", ["quadratic", "quartic"])
def test_proposition_2_1_graver_augmentation_is_globally_optimal(kind):
    A, b, l, u, x0 = _tiny()
    G = graver_basis_in_box(A, int(2 * (u - l).max()))
    F = np.array(sorted({canonical(g) for g in G}), dtype=np.int64)
    rng = np.random.default_rng(1 if kind == "quadratic" else 2)
    if kind == "quadratic":
        t = rng.integers(-2, 3, size=5)
        f = Objective("quadratic", Q=np.eye(5), c=(-2.0 * t).astype(float))
    else:
        coef = np.zeros((5, 5))
        coef[:, 4] = rng.integers(1, 3, size=5)
        coef[:, 2] = rng.integers(1, 4, size=5)
        coef[:, 1] = rng.integers(-6, 7, size=5)
        f = Objective("separable_poly", coef=coef)
    S = _feasible_points(A, b, l, u)
    fstar = min(_exact_f(f, x) for x in S)
    starts = np.array([S[i] for i in rng.choice(len(S), size=min(12, len(S)), replace=False)])
    X, fv, st, best = augment(A, b, l, u, f, F, starts)
    for x in X:
        assert _exact_f(f, x) == fstar


def test_augmentation_monotone_feasible_and_locally_optimal():
    inst = W.tiny_instance(1000)
    G = graver_basis_in_box(inst.A, 4)
    F = np.array(sorted({canonical(g) for g in G}), dtype=np.int64)
    f = Objective("quadratic", Q=inst.Q, c=inst.c)
    aug = Augmenter(f, F, inst.l, inst.u)
    x = inst.x0.copy()
    prev = _exact_f(f, x)
    while True:
        mv = aug.best_move(x)
        if mv is None or not mv[0] < 0:
            break
        _, pos, lam = mv
        g = F[pos // 2] * (1 if pos % 2 == 0 else -1)
        x = x + lam * g
        assert np.all(inst.A @ x == inst.b) and np.all(x >= inst.l) and np.all(x <= inst.u)
        cur = _exact_f(f, x)
        assert cur < prev
        # the chosen move is a true argmin over all (g, lam) pairs
        prev = cur
    # no improving (g, lam) at exit, checked exhaustively in exact arithmetic
    for g in np.concatenate([F, -F]):
        for lam in range(1, 11):
            y = x + lam * g
            if np.all(y >= inst.l) and np.all(y <= inst.u):
                assert _exact_f(f, y) >= _exact_f(f, x)


def test_best_move_is_exact_argmin_with_tie_rule():
    inst = W.tiny_instance(1000)
    G = graver_basis_in_box(inst.A, 3)
    F = np.array(sorted({canonical(g) for g in G}), dtype=np.int64)
    f = Objective("quadratic", Q=inst.Q, c=inst.c)
    aug = Augmenter(f, F, inst.l, inst.u)
    x = inst.x0
    fx = _exact_f(f, x)
    best = None
    for pos in range(2 * F.shape[0]):
        g = F[pos // 2] * (1 if pos % 2 == 0 else -1)
        for lam in range(1, 11):
            y = x + lam * g
            if np.all(y >= inst.l) and np.all(y <= inst.u):
                c = (_exact_f(f, y) - fx, pos, lam)
                best = c if best is None or c < best else best
    mv = aug.best_move(x)
    assert (Fraction(mv[0]), mv[1], mv[2]) == best


def test_infeasible_start_rejected_and_empty_set():
    A, b, l, u, x0 = _tiny()
    f = Objective("quadratic", Q=np.eye(5), c=np.zeros(5))
    with pytest.raises(ValueError):
        augment(A, b, l, u, f, np.zeros((0, 5), np.int64), [x0 + 1])
    X, fv, st, best = augment(A, b, l, u, f, np.zeros((0, 5), np.int64), [x0])
    assert np.array_equal(X[0], x0) and st[0] == 0

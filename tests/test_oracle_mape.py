"""Pins of the MAPE composition oracle (Section 3.3)."""
import itertools

import numpy as np
import pytest

from oracle import augment as AG
from oracle import conformal, lattice, mape
from oracle import surrogate as S
from paper_2412_13576_amd import workloads as W


def _tiny():
    inst = W.tiny_instance(1000)
    B = lattice.kernel_basis(inst.A)
    P = lattice.coordinate_projector(B)
    return inst, B, P


PRM = mape.MapeParams(n_starts=256, iters=300, seed=5, first_start=0, init_starts=64, init_iters=300,
                      init_seed=9, init_first_start=0, init_lr=0.05)


def test_mape_result_is_feasible_monotone_and_locally_optimal():
    inst, B, P = _tiny()
    f = AG.Objective("quadratic", Q=inst.Q, c=inst.c)
    r = mape.solve(inst.A, inst.b, inst.l, inst.u, f, B, P, PRM)
    x = r["x_best"]
    assert np.all(inst.A @ x == inst.b) and np.all((x >= inst.l) & (x <= inst.u))
    assert r["f_best"] == AG.objective(f, x)
    # every end point is no worse than its start, the best is the minimum
    for s in range(r["starts"].shape[0]):
        assert r["f"][s] <= AG.objective(f, r["starts"][s])
    assert r["f_best"] == min(r["f"])
    # no move along +-F improves the answer (Algorithm 1 stops there)
    F = np.array(r["F"], dtype=np.int64)
    fx = AG.objective(f, x)
    for g in F:
        for sg in (1, -1):
            for lam in range(1, 11):
                y = x + sg * lam * g
                if np.all((y >= inst.l) & (y <= inst.u)):
                    assert AG.objective(f, y) >= fx


def test_mape_with_graver_basis_reaches_global_optimum_separable_convex():
    """With the full Graver basis in place of the extracted set and a
    separable convex objective, every feasible start reaches the global
    optimum (Proposition 2.1); checked against enumeration of the box."""
    A = np.array([[1, 2, 1]], dtype=np.int64)
    b = np.array([4], dtype=np.int64)
    l = np.full(3, -3, np.int64)
    u = np.full(3, 3, np.int64)
    coef = np.array([[0.0, -1.3, 0.7], [0.0, 0.4, 1.1], [0.0, 2.0, 0.5]])
    f = AG.Objective("separable_poly", coef=coef)
    Gr = conformal.graver_basis_in_box(A, 6)
    from oracle import init_sol as I
    x0 = I.box_uniform_starts(l, u, 40, 3)
    _, R, feas = I.init_solutions(A, b, l, u, x0, 400, S.AdamParams(lr=0.05), 0.1)
    assert feas.any()
    X, fv, _, best = AG.augment(A, b, l, u, f, np.array(Gr, dtype=np.int64), R[feas])
    pts = [np.array(p) for p in itertools.product(range(-3, 4), repeat=3) if np.dot(A[0], p) == b[0]]
    opt = min(AG.objective(f, p) for p in pts)
    assert np.allclose(fv, opt, rtol=0, atol=1e-12)


def test_mape_no_feasible_start_raises():
    inst, B, P = _tiny()
    f = AG.Objective("quadratic", Q=inst.Q, c=inst.c)
    prm = mape.MapeParams(n_starts=8, iters=5, seed=1, first_start=0, init_starts=2, init_iters=0,
                          init_seed=1, init_first_start=0)
    with pytest.raises(ValueError):
        mape.solve(inst.A, inst.b + 1000, inst.l, inst.u, f, B, P, prm)

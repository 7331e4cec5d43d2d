"""Pins for the brute-force Graver basis and the minimality filter
(Section 1 definitions, condition C3)."""
import itertools

import numpy as np
import pytest

from oracle.conformal import (canonical, conformal_le, graver_basis_in_box, in_kernel,
                              kernel_vectors_in_box)
from oracle.minimal import filter_minimal, has_witness
from tests.golden_io import graver_closed_forms

CLOSED = graver_closed_forms()


@pytest.mark.parametrize("name,A,R,G", CLOSED, ids=[c[0] for c in CLOSED])
def test_brute_force_matches_closed_forms(name, A, R, G):
    got = graver_basis_in_box(A, R)
    want = sorted(set(G) | {tuple(-x for x in g) for g in G})
    assert got == want


def test_kernel_enumeration_is_complete_on_a_tiny_box():
    A = np.array([[1, 2, -1], [0, 1, 1]])
    R = 3
    brute = [g for g in itertools.product(range(-R, R + 1), repeat=3)
             if any(g) and in_kernel(A, g)]
    got = sorted(tuple(int(x) for x in g) for g in kernel_vectors_in_box(A, R))
    assert got == sorted(brute)


def test_brute_force_definition_on_random_matrix():
    rng = np.random.default_rng(5)
    A = rng.integers(-2, 3, size=(1, 4))
    while np.all(A == 0):
        A = rng.integers(-2, 3, size=(1, 4))
    R = 3
    Gb = set(graver_basis_in_box(A, R))
    allk = [g for g in itertools.product(range(-R, R + 1), repeat=4) if any(g) and in_kernel(A, g)]
    for g in allk:
        minimal = not any(h != g and conformal_le(h, g) for h in allk)
        assert minimal == (g in Gb)


def _kernel_pool(A, R):
    return [tuple(int(x) for x in g) for g in kernel_vectors_in_box(A, R)]


@pytest.mark.parametrize("name,A,R,G", CLOSED, ids=[c[0] for c in CLOSED])
def test_filter_recovers_graver_from_kernel_box(name, A, R, G):
    pool = _kernel_pool(A, R)
    out = filter_minimal(pool)
    assert out == sorted({canonical(g) for g in G})


def test_filter_invariants_random():
    rng = np.random.default_rng(11)
    A = np.array([[1, 1, 2, -1, 0], [0, 1, -1, 1, 2]])
    pool = _kernel_pool(A, 3)
    X = [pool[i] for i in rng.choice(len(pool), size=min(300, len(pool)), replace=False)]
    out = filter_minimal(X)
    Xs = {tuple(x) for x in X} | {tuple(-v for v in x) for x in X}
    # subset of +-input, canonical, antichain
    assert all(g in Xs for g in out)
    assert all(g == canonical(g) for g in out)
    C = np.array(out)
    for g in out:
        assert not has_witness(C, g)
    # every removed element has a witness in the input
    Xa = np.array(sorted({canonical(x) for x in X}))
    kept = set(out)
    for g in {canonical(x) for x in X}:
        if g not in kept:
            assert has_witness(Xa, g)
    # every Graver element present in the input survives
    Gb = {canonical(g) for g in graver_basis_in_box(A, 3)}
    assert {canonical(x) for x in X if canonical(x) in Gb} <= kept
    # idempotent, permutation and sign invariant
    assert filter_minimal(out) == out
    perm = [X[i] for i in rng.permutation(len(X))]
    flip = [tuple(-v for v in x) if rng.random() < 0.5 else x for x in perm]
    assert filter_minimal(flip) == out


def test_filter_edge_cases():
    assert filter_minimal([]) == []
    assert filter_minimal([(0, 0, 0)]) == []
    assert filter_minimal([(1, -1), (-1, 1), (1, -1)]) == [(1, -1)]
    # (1,0,-1) lies conformally below (2,0,-2) and (1,1,-2); (0,1,-1) below (1,1,-2)
    assert filter_minimal([(2, 0, -2), (1, 0, -1), (1, 1, -2), (0, -1, 1)]) == [(0, 1, -1), (1, 0, -1)]


def test_golden_tiny_graver_is_consistent():
    from tests.golden_io import tiny_graver_box6
    from paper_2412_13576_amd import workloads as W
    gold = tiny_graver_box6()
    assert sorted(gold) == list(range(1000, 1005))
    for seed, G in gold.items():
        A = W.tiny_instance(seed).A
        for g in list(G)[:200]:
            assert tuple(-x for x in g) in G and in_kernel(A, g)


def test_filter_closed_form_antichain_plus_conformal_sums():
    """Atoms on distinct supports of one size form an antichain; a sum of two
    sign-compatible atoms has the atom below it, so the minimal set is the
    atoms themselves (one per sign pair)."""
    from paper_2412_13576_amd.workloads import antichain_with_sums
    X, atoms = antichain_with_sums(n=12, n_atoms=40, support=3, n_sums=200, seed=3)
    got = filter_minimal([tuple(int(v) for v in r) for r in X])
    assert got == sorted({canonical(a) for a in atoms})

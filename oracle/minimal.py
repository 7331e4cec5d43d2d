"""Minimality filter with deduplication -- oracle, test infrastructure only.

Condition C3 of Section 3 asks for conformally minimal directions, and the
Graver basis (Section 1) is closed under negation.  Algorithm 2 collects
candidates without enforcing C3; this filter enforces it on the collected
set:

  1. C = the distinct elements of X union (-X);
  2. g in C survives iff no h in C with h != g satisfies h <= g
     (h_i g_i >= 0 and |h_i| <= |g_i| for all i);
  3. one representative per pair {g, -g} is returned (first nonzero entry
     positive), sorted lexicographically (signed, component 0 first).
"""
from __future__ import annotations

from typing import Iterable, List, Sequence, Tuple

import numpy as np

from .conformal import canonical


def filter_minimal(X: Iterable[Sequence[int]]) -> List[Tuple[int, ...]]:
    """Steps 1-3 above, written out directly (O(K^2) comparisons)."""
    C = set()
    for g in X:
        t = tuple(int(v) for v in g)
        if any(t):
            C.add(t)
            C.add(tuple(-v for v in t))
    Cl = sorted(C)
    if not Cl:
        return []
    V = np.array(Cl, dtype=np.int64)
    aV = np.abs(V)
    keep = []
    for k in range(V.shape[0]):
        g = V[k]
        below = np.all((V * g[None, :] >= 0) & (aV <= np.abs(g)[None, :]), axis=1)
        below[k] = False
        if not np.any(below):
            keep.append(canonical(Cl[k]))
    return sorted(set(keep))


def has_witness(C: np.ndarray, g: Sequence[int]) -> bool:
    """True iff some row h of C (or its negation), h != g, lies conformally
    below g.  C holds one representative per sign pair."""
    g = np.asarray(g, dtype=np.int64)
    ag = np.abs(g)
    for sgn in (1, -1):
        H = sgn * C
        below = np.all((H * g[None, :] >= 0) & (np.abs(H) <= ag[None, :]), axis=1)
        below &= np.any(H != g[None, :], axis=1)
        if np.any(below):
            return True
    return False

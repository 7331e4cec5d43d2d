"""Linear inequalities G x >= h (Section 3.4, eq. NLIP_ineq_slack and the
corollary after it) -- oracle, test infrastructure only.

With slacks s = G x - h >= 0 the program becomes one with equality
constraints only, over (x, s):
    [A 0; G -I] (x, s) = (b, h),  l <= x <= u,  0 <= s <= s_max,
and its integer kernel is the lattice of [B; G B] for a kernel basis B of
A (the corollary).  The surrogate over that basis has the extra term
||G B z||_1 (eq. surrogate_ineq) and is the plain surrogate of the lifted
program.  Reading (listed in the design notes): the slack upper bound
s_max_i = sum_j max(G_ij l_j, G_ij u_j) - h_i is the largest slack any x in
the box can have, so it removes no feasible point; it gives the slack rows
the same box condition C4 as the other coordinates.
"""
from __future__ import annotations

import numpy as np


def slack_bounds(G, h, l, u):
    G = np.asarray(G, dtype=object)
    smax = []
    for i in range(G.shape[0]):
        t = 0
        for j in range(G.shape[1]):
            t += max(int(G[i, j]) * int(l[j]), int(G[i, j]) * int(u[j]))
        smax.append(t - int(h[i]))
    return np.array(smax, dtype=np.int64)


def lift(A, b, l, u, G, h):
    """(A', b', l', u') of the slack form."""
    A = np.asarray(A, dtype=np.int64)
    G = np.asarray(G, dtype=np.int64)
    m, n = A.shape
    mi = G.shape[0]
    top = np.concatenate([A, np.zeros((m, mi), np.int64)], axis=1)
    bot = np.concatenate([G, -np.eye(mi, dtype=np.int64)], axis=1)
    A2 = np.concatenate([top, bot], axis=0)
    b2 = np.concatenate([np.asarray(b, np.int64), np.asarray(h, np.int64)])
    l2 = np.concatenate([np.asarray(l, np.int64), np.zeros(mi, np.int64)])
    u2 = np.concatenate([np.asarray(u, np.int64), slack_bounds(G, h, l, u)])
    return A2, b2, l2, u2


def lift_basis(B, G):
    """[B; G B] (exact integer product)."""
    B = np.asarray(B, dtype=object)
    G = np.asarray(G, dtype=object)
    return np.concatenate([B, G.dot(B)], axis=0).astype(np.int64)


def lift_point(x, G, h):
    """(x, G x - h)."""
    x = np.asarray(x, dtype=np.int64)
    return np.concatenate([x, np.asarray(G, np.int64) @ x - np.asarray(h, np.int64)])

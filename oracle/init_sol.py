"""Initial feasible solutions (Section 3.3, eq. init_sol) -- oracle, test
infrastructure only.

Starting points for the multi-start augmentation are found by minimising

    ||A x - b||_2^2 + lam3 * sum_i (x_i - floor x_i)(ceil x_i - x_i)

over x in the box [l, u] with Adam from many starting points, then rounding.
Readings where the paper is silent (listed with reasons in the design notes):
  * the box constraint is enforced by projection (clipping) after every Adam
    step;
  * starting points are uniform in [l, u] per component (Philox4x32-10, the
    same counter scheme as the extraction starts, or supplied by the caller);
  * lam3 = 0.1 (Section 4.1.2), Adam as in the extraction;
  * the paper states that optimal solutions are feasible; a rounded point
    is kept only when A x = b holds exactly and l <= x <= u.

binary64, ascending sums from 0.0, no fused multiply-add:
    res_i  = (sum_j A_ij x_j) - b_i
    grad_j = 2 * (sum_i A_ij res_i) + lam3 * ((ceil x_j + floor x_j) - 2 x_j)
"""
from __future__ import annotations

import numpy as np

from .philox import uniform01
from .surrogate import AdamParams, adam_step


def grad_init(A, b, x, lam3):
    """Gradient of eq. init_sol at each row of x (N, n)."""
    Af = np.asarray(A, dtype=np.float64)
    bf = np.asarray(b, dtype=np.float64)
    N, n = x.shape
    m = Af.shape[0]
    res = np.zeros((N, m))
    for j in range(n):
        res = res + Af[:, j][None, :] * x[:, j][:, None]
    res = res - bf[None, :]
    g = np.zeros((N, n))
    for i in range(m):
        g = g + Af[i, :][None, :] * res[:, i][:, None]
    t = np.ceil(x) + np.floor(x)
    t = t - 2.0 * x
    return 2.0 * g + lam3 * t


def objective_init(A, b, x, lam3):
    Af = np.asarray(A, dtype=np.float64)
    r = x @ Af.T - np.asarray(b, dtype=np.float64)[None, :]
    return (r * r).sum(axis=1) + lam3 * ((x - np.floor(x)) * (np.ceil(x) - x)).sum(axis=1)


def box_uniform_starts(l, u, n_starts, seed, first_start=0):
    """x0 uniform in [l, u] per component: l + U * (u - l)."""
    l = np.asarray(l, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    U = uniform01(n_starts, l.shape[0], seed, first_start)
    return l[None, :] + U * (u - l)[None, :]


def init_solutions(A, b, l, u, x0, iters, p: AdamParams, lam3=0.1):
    """Projected Adam from x0 (N, n), then rounding and the exact check.

    Returns (x_final, rounded (N, n) int64, feasible (N,) bool)."""
    lf = np.asarray(l, dtype=np.float64)
    uf = np.asarray(u, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    m = np.zeros_like(x)
    v = np.zeros_like(x)
    for t in range(1, iters + 1):
        g = grad_init(A, b, x, lam3)
        x, m, v = adam_step(x, m, v, g, t, p)
        x = np.minimum(np.maximum(x, lf[None, :]), uf[None, :])
    r = np.rint(x).astype(np.int64)
    A = np.asarray(A, dtype=np.int64)
    feas = np.all(r @ A.T == np.asarray(b)[None, :], axis=1)
    feas &= np.all(r >= np.asarray(l)[None, :], axis=1) & np.all(r <= np.asarray(u)[None, :], axis=1)
    return x, r, feas

"""Surrogate Phi, its gradient, Adam, and Parallel Extraction -- oracle,
test infrastructure only.

Follows Section 3.2: eq. loss

    Phi(z) = ||B z||_1 + lam1 * sum_i (z_i - floor z_i)(ceil z_i - z_i)
             + lam2 * max{ 1/||z||_inf - 1, 0 },

the Adam update (Kingma and Ba, the optimiser named in Section 3.2, with the
learning rate of Section 4.1.2), and Algorithm 2 (Parallel Extraction):
after every update t = 1..T the iterate is rounded, mapped to B round(z), and
kept when it lies in the box [l - u, u - l].

Readings where the paper is silent (each one is listed with its reason in
the design notes):
  * sign(0) = 0 as the subgradient of |.| at 0;
  * floor / ceil have zero derivative, so the integrality term has gradient
    lam1 * (ceil z + floor z - 2 z) (zero at integers);
  * the barrier term is differentiated only where 0 < ||z||_inf < 1, and its
    gradient is split evenly over the coordinates that attain the max;
  * rounding to the nearest integer breaks ties to even;
  * the zero vector is not collected (Algorithm 2 collects nonzero kernel
    elements);
  * Adam's beta1, beta2, eps are 0.9, 0.999, 1e-8; the loss is the sum over
    starts, so every start evolves independently;
  * a coordinate with |z_j| >= 2^30 makes that iterate yield no candidate.

Every floating-point formula below is evaluated in IEEE binary64 with the
operation order written in the code and no fused multiply-add; sums over an
index run in ascending order starting from 0.0.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Set, Tuple

import numpy as np

@dataclass
class AdamParams:
    lr: float = 0.003
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    lambda1: float = 0.85
    lambda2: float = 1.0


def phi(B: np.ndarray, z: np.ndarray, lam1: float, lam2: float) -> np.ndarray:
    """Phi(z) for every row of z (eq. loss).  z: (N, d) -> (N,)."""
    Bf = np.asarray(B, dtype=np.float64)
    y = z @ Bf.T
    l1 = np.abs(y).sum(axis=1)
    frac = ((z - np.floor(z)) * (np.ceil(z) - z)).sum(axis=1)
    mu = np.abs(z).max(axis=1)
    with np.errstate(divide="ignore"):
        bar = np.maximum(1.0 / mu - 1.0, 0.0)
    return l1 + lam1 * frac + lam2 * bar


def forward(Bf: np.ndarray, z: np.ndarray) -> np.ndarray:
    """y = B z per start, y_i = sum_j B_ij z_j in ascending j.  (N, n)."""
    N = z.shape[0]
    n, d = Bf.shape
    y = np.zeros((N, n))
    for j in range(d):
        y = y + Bf[:, j][None, :] * z[:, j][:, None]
    return y


def grad_phi(Bf: np.ndarray, z: np.ndarray, lam1: float, lam2: float) -> np.ndarray:
    """A (sub)gradient of Phi at each row of z.  (N, d) -> (N, d).

    grad = B^T sign(B z) + lam1 * ((ceil z + floor z) - 2 z) + barrier, where
    the barrier part is -lam2 * sign(z_k) / ((mu * mu) * c) at each of the c
    coordinates k with |z_k| = mu = ||z||_inf, applied when 0 < mu < 1.
    """
    N, d = z.shape
    n = Bf.shape[0]
    s = np.sign(forward(Bf, z))
    gb = np.zeros((N, d))
    for i in range(n):
        gb = gb + s[:, i][:, None] * Bf[i, :][None, :]
    t = np.ceil(z) + np.floor(z)
    t = t - 2.0 * z
    g = gb + lam1 * t
    az = np.abs(z)
    mu = az.max(axis=1)
    active = (mu > 0.0) & (mu < 1.0)
    if np.any(active):
        at_max = az == mu[:, None]
        cnt = at_max.sum(axis=1).astype(np.float64)
        w = np.where(active, lam2 / np.where(active, (mu * mu) * cnt, 1.0), 0.0)
        g = g - np.where(at_max & active[:, None], np.sign(z) * w[:, None], 0.0)
    return g


def adam_step(z, m, v, g, t: int, p: AdamParams):
    """One Adam update at step t (1-based), elementwise:
        m <- b1 m + (1-b1) g ;  v <- b2 v + (1-b2) (g g)
        mhat = m / (1 - b1^t) ; vhat = v / (1 - b2^t)
        z <- z - (lr mhat) / (sqrt(vhat) + eps)
    """
    m = p.beta1 * m + (1.0 - p.beta1) * g
    v = p.beta2 * v + (1.0 - p.beta2) * (g * g)
    bc1 = 1.0 - p.beta1 ** t
    bc2 = 1.0 - p.beta2 ** t
    mhat = m / bc1
    vhat = v / bc2
    z = z - (p.lr * mhat) / (np.sqrt(vhat) + p.eps)
    return z, m, v


def descend(B, z0: np.ndarray, iters: int, p: AdamParams, m0=None, v0=None,
            t0: int = 0, record: Tuple[int, ...] = ()):
    """Run ``iters`` Adam steps on Phi from (z0, m0, v0) after ``t0`` earlier
    steps.  Returns (z, m, v, snapshots) with snapshots[t] = z after global
    step t for t in ``record``."""
    Bf = np.asarray(B, dtype=np.float64)
    z = np.array(z0, dtype=np.float64)
    m = np.zeros_like(z) if m0 is None else np.array(m0, dtype=np.float64)
    v = np.zeros_like(z) if v0 is None else np.array(v0, dtype=np.float64)
    snaps = {}
    for k in range(1, iters + 1):
        t = t0 + k
        g = grad_phi(Bf, z, p.lambda1, p.lambda2)
        z, m, v = adam_step(z, m, v, g, t, p)
        if t in record:
            snaps[t] = z.copy()
    return z, m, v, snaps


def round_half_even(z: np.ndarray) -> np.ndarray:
    """Nearest integer, ties to even (IEEE rint)."""
    return np.rint(z)


def candidate(B: np.ndarray, r: np.ndarray) -> np.ndarray:
    """g = B r in exact integers for integer coordinate rows r (N, d)."""
    Bi = np.asarray(B, dtype=np.int64)
    rmax = float(np.abs(r).max(initial=0.0))
    bound = int(np.abs(Bi).sum(axis=1).max(initial=0)) * int(rmax)
    if bound >= 2 ** 62:
        # exact Python integers (r holds integral binary64 values)
        rows = [[sum(int(Bi[i, j]) * int(row[j]) for j in range(Bi.shape[1]))
                 for i in range(Bi.shape[0])] for row in r]
        return np.array(rows, dtype=object)
    return r.astype(np.int64) @ Bi.T


def in_box(g: np.ndarray, l: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Condition C4: l - u <= g <= u - l componentwise, and g != 0."""
    lo = (l - u)[None, :]
    hi = (u - l)[None, :]
    ok = np.all(g >= lo, axis=1) & np.all(g <= hi, axis=1)
    return ok & np.any(g != 0, axis=1)


def extract(A, B, l, u, z0: np.ndarray, iters: int, p: AdamParams,
            m0=None, v0=None, t0: int = 0, check_kernel: bool = True):
    """Algorithm 2 (Parallel Extraction) over the starts z0 (N, d).

    After each update t = t0+1..t0+iters: r = round(z^t) (ties to even);
    g = B r exactly; g is collected when it is nonzero and inside
    [l - u, u - l].  Collected vectors must satisfy A g = 0 (condition C1);
    a failure means B is not a kernel basis and raises.  Iterates whose r
    did not change since the previous step give the same g again, so they
    are skipped without changing the result.

    Returns (keys, state) where keys is a sorted list of distinct tuples
    (lexicographic, signed, component 0 first) and state = (z, m, v).
    """
    Bf = np.asarray(B, dtype=np.float64)
    Bi = np.asarray(B, dtype=np.int64)
    A = np.asarray(A, dtype=np.int64)
    l = np.asarray(l, dtype=np.int64)
    u = np.asarray(u, dtype=np.int64)
    z = np.array(z0, dtype=np.float64)
    m = np.zeros_like(z) if m0 is None else np.array(m0, dtype=np.float64)
    v = np.zeros_like(z) if v0 is None else np.array(v0, dtype=np.float64)
    found: Set[tuple] = set()
    r_prev: Optional[np.ndarray] = None
    for k in range(1, iters + 1):
        t = t0 + k
        g = grad_phi(Bf, z, p.lambda1, p.lambda2)
        z, m, v = adam_step(z, m, v, g, t, p)
        r = round_half_even(z)
        changed = np.ones(z.shape[0], bool) if r_prev is None else np.any(r != r_prev, axis=1)
        r_prev = r
        rows = np.nonzero(changed)[0]
        if rows.size == 0:
            continue
        gs = candidate(Bi, r[rows])
        keep = in_box(gs, l, u)
        for row in np.asarray(gs)[keep]:
            key = tuple(int(x) for x in row)
            if check_kernel and key not in found:
                if any(sum(int(A[i, j]) * key[j] for j in range(len(key))) != 0
                       for i in range(A.shape[0])):
                    raise AssertionError("collected vector is not in Ker(A)")
            found.add(key)
    return sorted(found), (z, m, v)

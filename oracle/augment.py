"""Augmentation scheme and objective -- oracle, test infrastructure only.

Algorithm 1 (Augmentation Scheme): from a feasible x, repeatedly pick
(g, lam) with g in the direction set, lam a positive integer, x + lam g in S
and f(x + lam g) < f(x), minimising f(x + lam g); move x to x + lam g; stop
when no such pair exists.  MAPE (Section 3.3) runs this from every start in
S_0 and returns the best end point.

Readings where the paper is silent (listed with reasons in the design notes):
  * the direction set is D = F union -F, ordered as F (canonical order)
    with each element followed by its negation;
  * S is {x : A x = b, l <= x <= u}; since every direction is a kernel
    vector, x + lam g stays in S iff it stays in the box, so lam runs over
    1..lam_max(g) with lam_max(g) = min over the support of
    floor((u_i - x_i)/g_i) (g_i > 0) or floor((x_i - l_i)/(-g_i)) (g_i < 0);
  * f(x + lam g) < f(x) is decided on Delta(g, lam) = f(x + lam g) - f(x)
    evaluated in binary64 by a fixed formula with no fused multiply-add and
    ascending sums over the support of g:
      quadratic f = x^T Q x + c^T x (Q symmetric):
        r_i = c_i + 2 * (sum_j Q_ij x_j)            (all j, fresh every step)
        a_g = sum_{i in supp g} g_i r_i
        q_g = sum_{i in supp g} g_i * (sum_{j in supp g} Q_ij g_j)
        Delta = (lam * a_g) + ((lam * lam) * q_g)
      separable polynomial f = sum_i p_i(x_i), p_i by Horner from the top
      coefficient:
        Delta = sum_{i in supp g} ( p_i(x_i + lam g_i) - p_i(x_i) );
    for integer data every quantity is an exact integer below 2^53, so the
    test is exact;
  * the minimum Delta wins; ties go to the earlier position in D, then to
    the smaller lam;
  * a move is taken iff Delta < 0; at most ``max_steps`` moves are made.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np


@dataclass
class Objective:
    kind: str                       # "quadratic" | "separable_poly"
    Q: Optional[np.ndarray] = None  # (n, n) float64, symmetric
    c: Optional[np.ndarray] = None  # (n,)
    coef: Optional[np.ndarray] = None  # (n, deg+1), coef[i, k] multiplies x_i^k


def horner(coef_row: Sequence[float], t: float) -> float:
    """p(t) = sum_k coef[k] t^k by Horner from the highest coefficient."""
    p = float(coef_row[-1])
    for k in range(len(coef_row) - 2, -1, -1):
        p = p * t + float(coef_row[k])
    return p


def objective(f: Objective, x: Sequence[int]) -> float:
    """f(x) in binary64 with ascending sums and no fused multiply-add.

    quadratic: (sum_i x_i * (sum_j Q_ij x_j)) + (sum_i c_i x_i), each sum from
    0.0; separable polynomial: sum_i p_i(x_i)."""
    xf = [float(v) for v in x]
    n = len(xf)
    if f.kind == "quadratic":
        s1 = 0.0
        for i in range(n):
            t = 0.0
            for j in range(n):
                t = t + float(f.Q[i, j]) * xf[j]
            s1 = s1 + xf[i] * t
        s2 = 0.0
        for i in range(n):
            s2 = s2 + float(f.c[i]) * xf[i]
        return s1 + s2
    s = 0.0
    for i in range(n):
        s = s + horner(f.coef[i], xf[i])
    return s


def _supports(F: np.ndarray):
    """Padded ascending supports of the rows of F: (idx, val, mask)."""
    K = F.shape[0]
    nnz = (F != 0).sum(axis=1)
    w = int(nnz.max(initial=0))
    idx = np.zeros((K, max(w, 1)), np.int64)
    val = np.zeros((K, max(w, 1)), np.int64)
    mask = np.zeros((K, max(w, 1)), bool)
    for k in range(K):
        cols = np.nonzero(F[k])[0]
        idx[k, :cols.size] = cols
        val[k, :cols.size] = F[k, cols]
        mask[k, :cols.size] = True
    return idx, val, mask


def _lam_max(F: np.ndarray, x: np.ndarray, l: np.ndarray, u: np.ndarray) -> np.ndarray:
    """lam_max(g) for each row g of F (exact integers); 0 when g = 0."""
    big = np.iinfo(np.int64).max
    pos = F > 0
    neg = F < 0
    with np.errstate(divide="ignore", invalid="ignore"):
        up = np.where(pos, (u - x)[None, :] // np.where(pos, F, 1), big)
        dn = np.where(neg, (x - l)[None, :] // np.where(neg, -F, 1), big)
    lm = np.minimum(up.min(axis=1), dn.min(axis=1))
    lm[~np.any(F != 0, axis=1)] = 0
    return lm


class Augmenter:
    """Algorithm 1 over a fixed direction set F (rows, one per sign pair)."""

    def __init__(self, f: Objective, F, l, u):
        self.f = f
        self.F = np.asarray(F, dtype=np.int64).reshape(-1, len(l))
        self.l = np.asarray(l, dtype=np.int64)
        self.u = np.asarray(u, dtype=np.int64)
        self.idx, self.val, self.mask = _supports(self.F)
        self.valf = self.val.astype(np.float64)
        if f.kind == "quadratic":
            self.qg = self._quad_q()

    def _quad_q(self) -> np.ndarray:
        """q_g = sum_{i in supp} g_i * (sum_{j in supp} Q_ij g_j), ascending."""
        K, w = self.idx.shape
        Q = np.asarray(self.f.Q, dtype=np.float64)
        q = np.zeros(K)
        for a in range(w):
            t = np.zeros(K)
            for b in range(w):
                term = Q[self.idx[:, a], self.idx[:, b]] * self.valf[:, b]
                t = np.where(self.mask[:, b], t + term, t)
            q = np.where(self.mask[:, a], q + self.valf[:, a] * t, q)
        return q

    def _deltas(self, x: np.ndarray, lam: int, sign: int) -> np.ndarray:
        """Delta(sign * g, lam) for every row g of F."""
        K, w = self.idx.shape
        lf = float(lam)
        if self.f.kind == "quadratic":
            return (lf * (sign * self._a)) + ((lf * lf) * self.qg)
        s = np.zeros(K)
        for a in range(w):
            col = self.idx[:, a]
            xi = x[col]
            new = xi + lam * sign * self.val[:, a]
            term = self._poly(col, new) - self._poly(col, xi)
            s = np.where(self.mask[:, a], s + term, s)
        return s

    def _poly(self, col: np.ndarray, t: np.ndarray) -> np.ndarray:
        coef = np.asarray(self.f.coef, dtype=np.float64)
        tf = t.astype(np.float64)
        p = coef[col, -1]
        for k in range(coef.shape[1] - 2, -1, -1):
            p = p * tf + coef[col, k]
        return p

    def _prepare(self, x: np.ndarray):
        if self.f.kind == "quadratic":
            Q = np.asarray(self.f.Q, dtype=np.float64)
            c = np.asarray(self.f.c, dtype=np.float64)
            xf = x.astype(np.float64)
            n = x.shape[0]
            s = np.zeros(n)
            for j in range(n):
                s = s + Q[:, j] * xf[j]
            r = c + 2.0 * s
            K, w = self.idx.shape
            a = np.zeros(K)
            for k in range(w):
                a = np.where(self.mask[:, k], a + self.valf[:, k] * r[self.idx[:, k]], a)
            self._a = a

    def best_move(self, x: np.ndarray):
        """(Delta, position in D, lam) of the best move, or None if F is empty."""
        K = self.F.shape[0]
        if K == 0:
            return None
        self._prepare(x)
        lm_p = _lam_max(self.F, x, self.l, self.u)
        lm_n = _lam_max(-self.F, x, self.l, self.u)
        best = None
        L = int(max(lm_p.max(initial=0), lm_n.max(initial=0)))
        for lam in range(1, L + 1):
            for sign, lm in ((1, lm_p), (-1, lm_n)):
                ok = lm >= lam
                if not np.any(ok):
                    continue
                dl = self._deltas(x, lam, sign)
                rows = np.nonzero(ok)[0]
                vals = dl[rows]
                vmin = vals.min()
                pos = 2 * rows[vals == vmin] + (0 if sign == 1 else 1)
                cand = (float(vmin), int(pos.min()), lam)
                if best is None or (cand[0], cand[1], cand[2]) < best:
                    best = cand
        return best

    def run(self, x_start, max_steps: int = 10 ** 6):
        """Algorithm 1 from x_start: returns (x, steps, hit_cap)."""
        x = np.asarray(x_start, dtype=np.int64).copy()
        steps = 0
        while steps < max_steps:
            mv = self.best_move(x)
            if mv is None or not (mv[0] < 0.0):
                return x, steps, False
            _, pos, lam = mv
            g = self.F[pos // 2] * (1 if pos % 2 == 0 else -1)
            x = x + lam * g
            steps += 1
        return x, steps, True


def check_feasible(A, b, l, u, x) -> bool:
    A = np.asarray(A, dtype=np.int64)
    x = np.asarray(x, dtype=np.int64)
    return bool(np.all(A @ x == np.asarray(b)) and np.all(x >= l) and np.all(x <= u))


def augment(A, b, l, u, f: Objective, F, starts, max_steps: int = 10 ** 6):
    """MAPE's multi-start augmentation (Section 3.3): Algorithm 1 from every
    start.  Returns (X, fvals, steps, best_index); best = smallest f, ties to
    the lowest start index.  Raises ValueError on an infeasible start."""
    starts = np.asarray(starts, dtype=np.int64)
    aug = Augmenter(f, F, l, u)
    X = np.empty_like(starts)
    fv = np.empty(starts.shape[0])
    st = np.empty(starts.shape[0], np.int64)
    for s in range(starts.shape[0]):
        if not check_feasible(A, b, l, u, starts[s]):
            raise ValueError(f"start {s} is infeasible")
        x, k, _ = aug.run(starts[s], max_steps)
        X[s] = x
        fv[s] = objective(f, x)
        st[s] = k
    best = int(np.argmin(fv)) if fv.size else -1
    return X, fv, st, best

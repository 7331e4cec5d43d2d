"""MAPE end to end (Section 3.3) -- oracle, test infrastructure only.

The composition the paper describes, step by step:
  1. Parallel Extraction (Algorithm 2) from Philox starts z0 = P g,
     g ~ U(l - u, u - l);
  2. the minimality filter (condition C3) on the collected set;
  3. initial solutions (eq. init_sol): projected Adam from x0 ~ U(l, u),
     rounding, exact feasibility test;
  4. augmentation (Algorithm 1) with D = F u (-F) from every feasible
     rounded point, in the order found, then from feasible points the
     caller supplies; the answer is the end point with the smallest
     objective (ties to the lowest start index).
Readings (listed with reasons in the design notes): the augmentation starts
are exactly the feasible initial solutions, duplicates kept; no feasible
initial solution is an error.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import augment as AG
from . import init_sol as I
from . import minimal
from . import philox
from . import surrogate as S


@dataclass
class MapeParams:
    n_starts: int            # extraction starts N
    iters: int               # extraction Adam steps T
    seed: int                # Philox key of the extraction starts
    first_start: int
    init_starts: int         # initial-solution starting points
    init_iters: int
    init_seed: int
    init_first_start: int
    init_lr: float = 0.003
    lambda3: float = 0.1
    max_steps: int = 10 ** 6


def solve(A, b, l, u, f: AG.Objective, B, P, prm: MapeParams, adam: S.AdamParams = S.AdamParams(),
          x_starts=None):
    """Returns a dict with the collected set, F, the feasible starts, every
    end point and objective value, and the best index."""
    _, z0 = philox.box_starts(P, l, u, prm.n_starts, seed=prm.seed, first_start=prm.first_start)
    keys, _ = S.extract(A, B, l, u, z0, prm.iters, adam)
    F = minimal.filter_minimal(keys)
    x0 = I.box_uniform_starts(l, u, prm.init_starts, prm.init_seed, prm.init_first_start)
    ip = S.AdamParams(lr=prm.init_lr, beta1=adam.beta1, beta2=adam.beta2, eps=adam.eps)
    _, R, feas = I.init_solutions(A, b, l, u, x0, prm.init_iters, ip, prm.lambda3)
    starts = R[feas]
    if x_starts is not None:
        starts = np.concatenate([starts, np.asarray(x_starts, dtype=np.int64).reshape(-1, R.shape[1])])
    if starts.shape[0] == 0:
        raise ValueError("no initial solution is feasible and no starts were given")
    Fa = np.array(F, dtype=np.int64).reshape(len(F), np.asarray(A).shape[1])
    X, fv, steps, best = AG.augment(A, b, l, u, f, Fa, starts, prm.max_steps)
    return dict(keys=keys, F=F, starts=starts, X=X, f=fv, steps=steps, best=best,
                x_best=X[best], f_best=float(fv[best]))

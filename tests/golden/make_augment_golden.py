"""Writes the stored augmentation results under tests/golden/ that come from
the oracle: Algorithm 1 from every start (MAPE's multi-start augmentation,
Section 3.3) on two synthetic cases large enough to span several direction
blocks and start groups of the device kernel:

  augment_qp_n100.txt       QP workload (m = 20, n = 100, nonconvex dense
                            quadratic, box [-10, 10]); 40000 sparse basis
                            combinations with |g_i| <= 20 (about 25000
                            directions); 48 feasible-walk starts
  augment_quartic_n400.txt  quartic workload (m = 50, n = 400, separable
                            degree-4 polynomial, box [-20, 20]); 1500
                            combinations with |g_i| <= 40; 33 starts

Inputs come from the seeded generators (paper_2412_13576_amd.workloads) and
the oracle's kernel basis; results from oracle.augment.augment, one process
per group of starts (each start's run is independent).  Each file records a
SHA-256 of the direction set and the starts so a reader can confirm it
regenerated the same inputs.  Run from the repository root:
    python tests/golden/make_augment_golden.py
"""
import hashlib
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import lattice  # noqa: E402
from oracle.augment import Objective, augment  # noqa: E402
from paper_2412_13576_amd import workloads as W  # noqa: E402

CASES = {
    "qp": dict(file="augment_qp_n100.txt", count=40000, density=0.05, limit=20, starts=48, seed=41),
    "quartic": dict(file="augment_quartic_n400.txt", count=1500, density=0.01, limit=40, starts=33, seed=43),
}


def case_inputs(kind):
    """(instance, objective, directions F, starts) of one case."""
    c = CASES[kind]
    inst = W.qp_instance(2000) if kind == "qp" else W.quartic_instance(3000)
    B = lattice.kernel_basis(inst.A)
    F = W.combination_directions(B, c["count"], c["density"], c["limit"], c["seed"])
    starts = W.feasible_walk_starts(inst.x0, F, inst.l, inst.u, c["starts"], seed=c["seed"] + 1, walk_len=16)
    f = Objective("quadratic", Q=inst.Q, c=inst.c) if kind == "qp" else Objective("separable_poly", coef=inst.coef)
    return inst, f, F, starts


def inputs_sha256(F, starts):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(F, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(starts, dtype=np.int64).tobytes())
    return h.hexdigest()


def _run(args):
    kind, lo, hi = args
    inst, f, F, starts = case_inputs(kind)
    X, fv, st, _ = augment(inst.A, inst.b, inst.l, inst.u, f, F, starts[lo:hi])
    return lo, X, fv, st


def write(kind, procs):
    c = CASES[kind]
    inst, f, F, starts = case_inputs(kind)
    S = starts.shape[0]
    chunks = [(kind, lo, min(S, lo + 2)) for lo in range(0, S, 2)]
    with mp.get_context("spawn").Pool(procs) as pool:
        parts = pool.map(_run, chunks)
    X = np.empty_like(starts)
    fv = np.empty(S)
    st = np.empty(S, np.int64)
    for lo, Xp, fp, sp in parts:
        X[lo:lo + Xp.shape[0]] = Xp
        fv[lo:lo + Xp.shape[0]] = fp
        st[lo:lo + Xp.shape[0]] = sp
    best = int(np.argmin(fv))
    path = os.path.join(HERE, c["file"])
    with open(path, "w") as fh:
        fh.write(f"# Algorithm 1 from every start (oracle.augment.augment), case '{kind}', written by\n")
        fh.write("# make_augment_golden.py.  Per start: index, moves, f(x_end) as binary64 bits (hex),\n")
        fh.write("# then x_end.\n")
        fh.write(f"inputs {inputs_sha256(F, starts)} K {F.shape[0]} S {S} n {inst.n} best {best}\n")
        for s in range(S):
            bits = np.array([fv[s]]).view(np.uint64)[0]
            fh.write(f"{s} {st[s]} {bits:016x} " + " ".join(str(int(v)) for v in X[s]) + "\n")
    print("wrote", path, "K", F.shape[0], "S", S, "moves", int(st.sum()))


if __name__ == "__main__":
    kinds = sys.argv[1:] or list(CASES)
    for k in kinds:
        write(k, min(8, os.cpu_count() or 1))

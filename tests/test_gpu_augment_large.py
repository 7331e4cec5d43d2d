"""Augmentation parity at sizes that span many 256-direction blocks and
several 16-start groups of the device kernel: graver_augment against stored
oracle results (tests/golden/augment_*.txt, written by
tests/golden/make_augment_golden.py from oracle.augment.augment), bit for
bit: every end point, move count, objective bits and the best index.

  qp       QP workload, about 25000 directions x 48 starts (3 groups), 812 moves
  quartic  quartic workload (separable degree-4 f), 1217 directions x 33
           starts (3 groups)
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from tests import golden_io  # noqa: E402
from make_augment_golden import CASES, case_inputs, inputs_sha256  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2412_13576_amd import graver
    return graver


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind", ["qp", "quartic"])
def test_augment_matches_oracle_golden(G, ctx, kind):
    sha, best_o, rows = golden_io.augment_golden(CASES[kind]["file"])
    inst, f, F, starts = case_inputs(kind)
    assert inputs_sha256(F, starts) == sha, "regenerated inputs differ from the fixture's"
    _say("augment golden", kind, "K", F.shape[0], "S", starts.shape[0])
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, np.zeros((inst.n, 1), np.int64))
    obj = G.objective(f.kind, Q=f.Q, c=f.c, coef=f.coef)
    x, fv, steps, best = G.augment(ctx, prob, obj, torch.tensor(F.astype(np.int8), device="cuda"),
                                   torch.tensor(starts, device="cuda"))
    x = x.cpu().numpy()
    fb = fv.cpu().numpy().view(np.uint64)
    st = steps.cpu().numpy()
    for s, (moves, bits, xe) in enumerate(rows):
        assert st[s] == moves, f"start {s}"
        assert np.array_equal(x[s], xe), f"start {s}"
        assert int(fb[s]) == bits, f"start {s}"
    assert best == best_o
    assert int(st.sum()) > 0

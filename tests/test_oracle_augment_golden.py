"""The stored augmentation fixtures (tests/golden/augment_*.txt) against the
oracle as it stands: their inputs regenerate to the recorded hash, and a
re-run of oracle.augment.augment on two of the QP case's starts reproduces
their rows bit for bit."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from tests import golden_io  # noqa: E402
from make_augment_golden import CASES, case_inputs, inputs_sha256  # noqa: E402

from oracle.augment import augment  # noqa: E402


def test_qp_fixture_reproduces():
    sha, best, rows = golden_io.augment_golden(CASES["qp"]["file"])
    inst, f, F, starts = case_inputs("qp")
    assert inputs_sha256(F, starts) == sha
    fv_all = np.array([r[1] for r in rows], np.uint64).view(np.float64)
    assert len(rows) == starts.shape[0] and best == int(np.argmin(fv_all))
    pick = [0, 5]
    X, fv, st, _ = augment(inst.A, inst.b, inst.l, inst.u, f, F, starts[pick])
    for k, s in enumerate(pick):
        moves, bits, xe = rows[s]
        assert st[k] == moves and np.array_equal(X[k], xe)
        assert int(np.array([fv[k]]).view(np.uint64)[0]) == bits
        assert moves > 0


def test_quartic_fixture_inputs():
    sha, best, rows = golden_io.augment_golden(CASES["quartic"]["file"])
    inst, f, F, starts = case_inputs("quartic")
    assert inputs_sha256(F, starts) == sha
    assert len(rows) == starts.shape[0] >= 33 and F.shape[0] > 512

"""Condition C1 (A g = 0) through graver_verify: kernel vectors pass, and
rows that are not kernel vectors are counted and reported as
GRAVER_E_NOT_KERNEL, in both device forms of the check (a thread per key
for a small A, a wave per key beyond 4096 nonzeros).  The expected counts
come from the oracle's exact check."""
import numpy as np
import pytest

from oracle import lattice
from oracle.conformal import in_kernel
from paper_2412_13576_amd import workloads as W

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


def _case(kind):
    if kind == "qp":  # 20 x 100, about 600 nonzeros: thread-per-key form
        inst = W.qp_instance(2000)
        B = lattice.kernel_basis(inst.A)
        F = W.combination_directions(B, 6000, 0.05, 20, 51)
    else:  # identity block 100 x 500, about 8100 nonzeros: wave-per-key form
        inst = W.identity_block_instance(52, 500, 100)
        m, n = inst.A.shape
        C = inst.A[:, m:]
        B = np.vstack([-C, np.eye(n - m, dtype=np.int64)])
        F = W.combination_directions(B, 3000, 0.01, 5, 53)
    return inst, F


@pytest.mark.parametrize("kind", ["qp", "wide"])
def test_verify_accepts_kernel_and_counts_violations(G, ctx, kind):
    inst, F = _case(kind)
    _say("verify", kind, F.shape, int((inst.A != 0).sum()))
    assert not np.any(inst.A @ F.T)  # every generated row is a kernel vector (exact int64)
    A = torch.tensor(inst.A, device="cuda")
    keys = torch.tensor(F.astype(np.int8), device="cuda")
    st, nb = G.verify(ctx, A, keys)
    assert (st, nb) == (0, 0)
    # perturb a seeded subset of rows by one unit in one coordinate
    rng = np.random.default_rng(7)
    bad = F.copy()
    rows = rng.choice(F.shape[0], size=37, replace=False)
    for r in rows:
        j = int(rng.integers(0, F.shape[1]))
        bad[r, j] += 1 if bad[r, j] < 100 else -1
    expect = sum(0 if in_kernel(inst.A, bad[r]) else 1 for r in rows)
    assert expect > 0
    st, nb = G.verify(ctx, A, torch.tensor(bad.astype(np.int8), device="cuda"))
    assert st == -3 and nb == expect
    # a single non-kernel row among kernel rows at the end of the last tile
    one = F.copy()
    one[-1] = 0
    one[-1, 0] = 1
    st, nb = G.verify(ctx, A, torch.tensor(one.astype(np.int8), device="cuda"))
    assert st == -3 and nb == (0 if in_kernel(inst.A, one[-1]) else 1) == 1
    st, nb = G.verify(ctx, A, keys[:0])
    assert (st, nb) == (0, 0)

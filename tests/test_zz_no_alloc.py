"""The allocation-free augmentation entry point (graver_augment_noalloc)
against graver_augment through the C ABI: identical iterates, step counts,
objective bits and best index, on two calls in a row (the second smaller, so
the shared device scratch holds the first call's data when it starts), for
a quadratic and a separable quartic objective; calls beyond the scratch
limit are refused."""
import numpy as np
import pytest

from oracle import lattice
from oracle.conformal import canonical
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
    """Directions that move interior starts: sparse integer combinations of
    the basis columns inside the box, and feasible-walk starts."""
    if kind == "qp":
        inst = W.qp_instance(2000)
        lim, p, S0 = 20, 0.05, 40
    else:
        inst = W.quartic_instance(3000)
        lim, p, S0 = 40, 0.01, 36
    B = lattice.kernel_basis(inst.A)
    rng = np.random.default_rng(17)
    Z = rng.integers(-1, 2, size=(3000, B.shape[1])) * (rng.random((3000, B.shape[1])) < p)
    G_ = Z @ B.T
    G_ = G_[np.all(np.abs(G_) <= lim, axis=1) & np.any(G_ != 0, axis=1)]
    F = np.array(sorted({canonical(g) for g in G_}), dtype=np.int64)
    starts = W.feasible_walk_starts(inst.x0, F, inst.l, inst.u, S0, seed=23, walk_len=16)
    return inst, F, starts


def _obj(G, kind, inst):
    if kind == "qp":
        return G.objective("quadratic", Q=inst.Q, c=inst.c)
    return G.objective("separable_poly", coef=inst.coef)


@pytest.mark.parametrize("kind", ["qp", "quartic"])
def test_noalloc_equals_augment_twice(G, ctx, kind):
    inst, F, starts = _case(kind)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, np.zeros((inst.n, 1), np.int64))
    obj = _obj(G, kind, inst)
    Fd = torch.tensor(F.astype(np.int8), device="cuda")
    Sd = torch.tensor(starts, device="cuda")
    # first call: every direction and start; second: fewer of both
    for K, S in ((F.shape[0], starts.shape[0]), (F.shape[0] // 3, starts.shape[0] // 2 + 1)):
        _say("noalloc", kind, "K", K, "S", S)
        ref = G.augment(ctx, prob, obj, Fd[:K], Sd[:S])
        got = G.augment(ctx, prob, obj, Fd[:K], Sd[:S], noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(got[0], ref[0])
        assert torch.equal(got[2], ref[2])
        assert np.array_equal(got[1].cpu().numpy().view(np.uint64), ref[1].cpu().numpy().view(np.uint64))
        assert got[3] == ref[3]
        assert int(ref[2].sum()) > 0  # the case makes moves


def test_noalloc_limits_and_errors(G, ctx):
    inst, F, starts = _case("qp")
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, np.zeros((inst.n, 1), np.int64))
    obj = _obj(G, "qp", inst)
    Sd = torch.tensor(starts, device="cuda")
    # more directions than the scratch array can cache: refused before any work
    big = torch.zeros((1 << 24, inst.n), dtype=torch.int8, device="cuda")
    with pytest.raises(G.GraverError) as e:
        G.augment(ctx, prob, obj, big, Sd, noalloc=True)
    assert e.value.status == -8
    del big
    Fd = torch.tensor(F.astype(np.int8), device="cuda")
    bad = starts.copy()
    bad[0, 0] += 1
    with pytest.raises(G.GraverError) as e:
        G.augment(ctx, prob, obj, Fd, torch.tensor(bad, device="cuda"), noalloc=True)
    assert e.value.status == -2
    Qa = inst.Q.copy()
    Qa[0, 1] += 1.0
    with pytest.raises(G.GraverError) as e:
        G.augment(ctx, prob, G.objective("quadratic", Q=Qa, c=inst.c), Fd, Sd, noalloc=True)
    assert e.value.status == -1
    # after the refusals a call still equals graver_augment
    ref = G.augment(ctx, prob, obj, Fd, Sd)
    got = G.augment(ctx, prob, obj, Fd, Sd, noalloc=True)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[2], ref[2]) and got[3] == ref[3]

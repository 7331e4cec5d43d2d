"""GPU parity of the end-to-end solve (MAPE, Section 3.3) against the
oracle composition, and the reuse of one extraction across instances that
share A and the box widths."""
import numpy as np
import pytest

from oracle import augment as AG
from oracle import lattice, mape
from paper_2412_13576_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2412_13576_amd import graver
    return graver


def _params(G, prm: mape.MapeParams, precision, reuse):
    ex = G.extract_params(prm.n_starts, prm.iters, precision=precision, init_mode=0, seed=prm.seed,
                          first_start=prm.first_start, pool_capacity=1 << 20)
    ini = G.init_params(prm.init_starts, prm.init_iters, init_mode=0, seed=prm.init_seed,
                        first_start=prm.init_first_start, lr=prm.init_lr, lambda3=prm.lambda3)
    return G.solve_params(ex, ini, max_steps=prm.max_steps, reuse=reuse)


PRM = mape.MapeParams(n_starts=1024, iters=500, seed=77, first_start=0, init_starts=128, init_iters=300,
                      init_seed=9, init_first_start=0, init_lr=0.05)


@pytest.mark.parametrize("with_x", [False, True], ids=["init-only", "init+x0"])
def test_solve_fp64_bit_exact_vs_oracle(G, with_x):
    inst = W.tiny_instance(1000)
    B = lattice.kernel_basis(inst.A)
    P = lattice.coordinate_projector(B)
    f = AG.Objective("quadratic", Q=inst.Q, c=inst.c)
    _say("solve fp64 tiny", with_x)
    xs = np.stack([inst.x0, inst.x0]) if with_x else None
    ref = mape.solve(inst.A, inst.b, inst.l, inst.u, f, B, P, PRM, x_starts=xs)
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    obj = G.objective("quadratic", Q=inst.Q, c=inst.c)
    sp = _params(G, PRM, G.GRAVER_FP64, reuse=False)
    if with_x:
        sp = G.solve_params(sp.extract, sp.init, max_steps=PRM.max_steps, reuse=False,
                            x_starts=torch.tensor(xs, device="cuda"))
    x, fb, st = G.solve(ctx, prob, obj, sp)
    _say("solve fp64 tiny", st, "oracle f", ref["f_best"])
    assert np.array_equal(x.cpu().numpy(), ref["x_best"])
    assert np.float64(fb).view(np.uint64) == np.float64(ref["f_best"]).view(np.uint64)
    assert st["unique"] == len(ref["keys"]) and st["filtered"] == len(ref["F"])
    assert st["feasible_starts"] + (2 if with_x else 0) == ref["starts"].shape[0]
    assert st["best_start"] == ref["best"] and st["augment_steps"] == int(ref["steps"].sum())
    ctx.close()


def test_solve_reuses_extraction_for_same_A(G):
    """A second instance with the same A and box (new b, new objective)
    reuses the cached set and gives the same answer as a fresh solve."""
    inst = W.tiny_instance(1000)
    B = lattice.kernel_basis(inst.A)
    P = lattice.coordinate_projector(B)
    x2 = np.array([1, -1, 0, 2, 0, -2, 1, 0], dtype=np.int64)
    b2 = inst.A @ x2
    c2 = np.arange(8, dtype=np.float64) - 3.5
    _say("solve reuse")
    ctx = G.Context(0)
    p1 = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    p2 = G.DeviceProblem.from_numpy(inst.A, b2, inst.l, inst.u, B, P)
    o1 = G.objective("quadratic", Q=inst.Q, c=inst.c)
    o2 = G.objective("quadratic", Q=inst.Q, c=c2)
    prm = _params(G, PRM, G.GRAVER_FP64, reuse=True)
    _, _, s1 = G.solve(ctx, p1, o1, prm)
    xa, fa, s2 = G.solve(ctx, p2, o2, prm)
    assert s1["reused"] == 0 and s2["reused"] == 1 and s2["filtered"] == s1["filtered"]
    fresh = G.Context(0)
    xb, fb, s3 = G.solve(fresh, p2, o2, _params(G, PRM, G.GRAVER_FP64, reuse=False))
    assert s3["reused"] == 0
    assert torch.equal(xa, xb) and fa == fb
    assert np.all(inst.A @ xa.cpu().numpy() == b2)
    _say("solve reuse", s1["ms_extract"], s2["ms_extract"], "f", fa)
    ctx.close()
    fresh.close()


def test_solve_library_basis_fp32_qp(G):
    """The library computes B and P itself (host HNF + LLL); binary32
    extraction on matrix cores; the answer is feasible and its objective is
    the oracle's objective of the returned point, bit for bit."""
    inst = W.qp_instance(2000)
    _say("solve qp fp32 library basis")
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, None)
    obj = G.objective("quadratic", Q=inst.Q, c=inst.c)
    prm = mape.MapeParams(n_starts=8192, iters=500, seed=3, first_start=0, init_starts=200, init_iters=500,
                          init_seed=4, init_first_start=0, init_lr=0.05)
    # the initial-solution search rarely rounds onto A x = b at this shape,
    # so the generator's feasible point joins the starts
    sp = _params(G, prm, G.GRAVER_FP32, reuse=True)
    xs = torch.tensor(inst.x0[None, :], device="cuda")
    sp = G.solve_params(sp.extract, sp.init, max_steps=prm.max_steps, reuse=True, x_starts=xs)
    x, fb, st = G.solve(ctx, prob, obj, sp)
    xh = x.cpu().numpy()
    _say("solve qp fp32", st, "f", fb)
    assert st["d"] == 80
    assert np.all(inst.A @ xh == inst.b) and np.all((xh >= inst.l) & (xh <= inst.u))
    f = AG.Objective("quadratic", Q=inst.Q, c=inst.c)
    assert np.float64(fb).view(np.uint64) == np.float64(AG.objective(f, xh)).view(np.uint64)
    assert fb <= AG.objective(f, inst.x0)
    ctx.close()


def test_solve_errors(G):
    inst = W.tiny_instance(1000)
    B = lattice.kernel_basis(inst.A)
    P = lattice.coordinate_projector(B)
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b + 1000, inst.l, inst.u, B, P)
    obj = G.objective("quadratic", Q=inst.Q, c=inst.c)
    prm = mape.MapeParams(n_starts=64, iters=10, seed=1, first_start=0, init_starts=8, init_iters=5,
                          init_seed=1, init_first_start=0)
    with pytest.raises(G.GraverError) as e:
        G.solve(ctx, prob, obj, _params(G, prm, G.GRAVER_FP64, reuse=False))
    assert e.value.status == G.GRAVER_E_INFEASIBLE_START
    ctx.close()

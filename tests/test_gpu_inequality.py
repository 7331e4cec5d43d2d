"""GPU parity on programs with linear inequalities (Section 3.4): the
slack form from the library's lift, the basis [B; G B], and the ordinary
descent, filter, augmentation and solve on it, against the oracle."""
import numpy as np
import pytest

from oracle import augment as AG
from oracle import inequality as Q
from oracle import lattice, mape
from oracle import surrogate as S
from paper_2412_13576_amd import workloads as W
from tests.test_gpu_fp32 import TOL, _check_step, _relerr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
P_ = S.AdamParams()


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


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _lifted(G, inst, mi, seed, mag=2):
    Gm, h = W.inequality_rows(inst, mi, seed, nnz=4, mag=mag)
    B = lattice.kernel_basis(inst.A)
    A2, b2, l2, u2 = Q.lift(inst.A, inst.b, inst.l, inst.u, Gm, h)
    Bt = Q.lift_basis(B, Gm)
    return Gm, h, A2, b2, l2, u2, Bt


def test_ineq_fp64_extract_bit_exact(G, ctx):
    inst = W.tiny_instance(1000)
    Gm, h, A2, b2, l2, u2, Bt = _lifted(G, inst, 2, 1)
    _say("ineq fp64 extract", A2.shape, Bt.shape, "slack bounds", u2[inst.n:].tolist())
    N, T = 1024, 500
    z0 = W.gaussian_starts(N, Bt.shape[1], 2.0, 31)
    prob = G.DeviceProblem.from_numpy(A2, b2, l2, u2, Bt)
    st = {"z": _dev(z0)}
    k, _ = G.extract(ctx, prob, G.extract_params(N, T, precision=G.GRAVER_FP64, init_mode=1,
                                                  pool_capacity=1 << 18), state=st)
    keys, (zo, _, _) = S.extract(A2, Bt, l2, u2, z0, T, P_)
    assert np.array_equal(st["z"].cpu().numpy().view(np.uint64), zo.view(np.uint64))
    got = sorted(tuple(r) for r in k.cpu().numpy().astype(np.int64).tolist())
    assert got == [tuple(x) for x in keys]
    # every candidate is (g, G g) with A g = 0
    K = np.array(got, dtype=np.int64)
    assert np.all(K[:, :inst.n] @ inst.A.T == 0) and np.all(K[:, :inst.n] @ Gm.T == K[:, inst.n:])
    _say("ineq fp64 extract", "keys", len(got))


def test_ineq_solve_fp64_vs_oracle(G):
    inst = W.tiny_instance(1000)
    Gm, h, A2, b2, l2, u2, Bt = _lifted(G, inst, 2, 1)
    P = lattice.coordinate_projector(Bt)
    mi = Gm.shape[0]
    Q2 = np.zeros((inst.n + mi, inst.n + mi))
    Q2[:inst.n, :inst.n] = inst.Q
    c2 = np.concatenate([inst.c, np.zeros(mi)])
    f = AG.Objective("quadratic", Q=Q2, c=c2)
    prm = mape.MapeParams(n_starts=1024, iters=500, seed=7, first_start=0, init_starts=128, init_iters=300,
                          init_seed=9, init_first_start=0, init_lr=0.05)
    _say("ineq solve fp64")
    x0 = Q.lift_point(inst.x0, Gm, h)[None, :]
    ref = mape.solve(A2, b2, l2, u2, f, Bt, P, prm, x_starts=x0)
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(A2, b2, l2, u2, Bt, P)
    obj = G.objective("quadratic", Q=Q2, c=c2)
    ex = G.extract_params(prm.n_starts, prm.iters, precision=G.GRAVER_FP64, init_mode=0, seed=prm.seed,
                          pool_capacity=1 << 20)
    ini = G.init_params(prm.init_starts, prm.init_iters, seed=prm.init_seed, lr=prm.init_lr)
    sp = G.solve_params(ex, ini, reuse=False, x_starts=torch.tensor(x0, device="cuda"))
    x, fb, st = G.solve(ctx, prob, obj, sp)
    xh = x.cpu().numpy()
    _say("ineq solve fp64", st, "f", fb, "oracle", ref["f_best"])
    assert np.array_equal(xh, ref["x_best"])
    assert np.float64(fb).view(np.uint64) == np.float64(ref["f_best"]).view(np.uint64)
    assert np.all(inst.A @ xh[:inst.n] == inst.b) and np.all(Gm @ xh[:inst.n] >= h)
    assert np.array_equal(xh[inst.n:], Gm @ xh[:inst.n] - h)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ineq_qp_matrix_core_parity(G, ctx, prec):
    """QP workload with 10 inequalities (n + m' = 110): binary32 / bf16
    steps from oracle states match the oracle, and the sets match the
    binary64 GPU set of the same starts."""
    inst = W.qp_instance(2000)
    Gm, h, A2, b2, l2, u2, Bt = _lifted(G, inst, 10, 2)
    _say("ineq qp", prec, Bt.shape, "slack bounds max", int(u2[inst.n:].max()))
    prob = G.DeviceProblem.from_numpy(A2, b2, l2, u2, Bt)
    precision = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
    N = 256
    z0 = W.gaussian_starts(N, Bt.shape[1], 2.0, 32)
    for t_teacher in (0, 40):
        z, mm, vv, _ = (S.descend(Bt, z0, t_teacher, P_) if t_teacher
                        else (z0, np.zeros_like(z0), np.zeros_like(z0), 0))
        zo, _, _, _ = S.descend(Bt, z, 1, P_, m0=mm, v0=vv, t0=t_teacher)
        st = {"z": _dev(z), "m": _dev(mm), "v": _dev(vv)}
        G.extract(ctx, prob, G.extract_params(N, 1, precision=precision, init_mode=1, t0=t_teacher, collect=0),
                  state=st)
        err, flagged = _check_step(Bt, z, mm, vv, t_teacher + 1, st["z"].cpu().numpy(), zo)
        _say("ineq qp", prec, t_teacher, "max err", float(err.max()), "kink starts", flagged)
    z1 = W.gaussian_starts(2048, Bt.shape[1], 0.3, 33)
    sets = {}
    for p in (G.GRAVER_FP64, precision):
        k, s = G.extract(ctx, prob, G.extract_params(2048, 80, precision=p, init_mode=1, pool_capacity=1 << 20),
                         state={"z": _dev(z1)})
        sets[p] = {tuple(r) for r in k.cpu().numpy().tolist()}
        K = k.cpu().numpy().astype(np.int64)
        assert np.all(K @ A2.T == 0) and np.all(np.abs(K) <= (u2 - l2)[None, :])
    a, b = sets[precision], sets[G.GRAVER_FP64]
    jac = len(a & b) / max(1, len(a | b))
    _say("ineq qp sets", prec, len(a), len(b), "jaccard", jac)
    assert len(b) > 0 and jac >= 0.9

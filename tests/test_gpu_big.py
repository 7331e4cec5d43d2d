"""GPU parity of the large-basis matrix-core descent (n > 128: the basis is
streamed through LDS one 16-row block at a time, and the exact candidate is
recomputed on bf16 operands) against the binary64 oracle and the binary64
GPU path.  Instances: A = [I_m | C] with sparse C (cheap exact kernel
basis at large n).  The binary32 calls name the matrix-core form (the
library's default on these sparse bases is the sparse form, which the
"fp32-sparse" cases cover)."""
import numpy as np
import pytest

from oracle import lattice
from oracle import surrogate as S
from paper_2412_13576_amd import workloads as W
from tests.test_gpu_fp32 import TOL, _check_step, _relerr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
P_ = S.AdamParams()

SHAPES = [(200, 40), (300, 60), (600, 450)]   # (n, m): d = 160, 240, 150


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


_cache = {}


def _inst(n, m):
    if (n, m) not in _cache:
        inst = W.identity_block_instance(5000 + n, n, m)
        B = lattice.kernel_basis(inst.A)
        P = lattice.coordinate_projector(B) if n <= 200 else None
        _cache[(n, m)] = (inst, B, P)
    return _cache[(n, m)]


def _row_list_entries(B):
    """Row-list entries per lane of the sparse form: rows by decreasing
    nonzero count in slots of 64, each slot as wide as its longest row."""
    cnt = np.sort((np.asarray(B) != 0).sum(axis=1))[::-1]
    return int(sum(cnt[i] for i in range(0, cnt.size, 64)))


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{n}" for n, _ in SHAPES])
@pytest.mark.parametrize("prec", ["fp32", "fp32-sparse", "bf16"])
def test_big_teacher_forced_single_step(G, ctx, shape, prec):
    n, m = shape
    inst, B, _ = _inst(n, m)
    _say("big teacher-forced", n, B.shape[1], prec)
    N = 50                          # ragged: the last wave holds 2 starts
    z0 = W.gaussian_starts(N, B.shape[1], 2.0, 77)
    if prec == "fp32-sparse" and _row_list_entries(B) > 128:
        # beyond the form's limit: the call is refused, nothing runs
        prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
        st = {"z": _dev(z0)}
        with pytest.raises(G.GraverError, match="sparse form"):
            G.extract(ctx, prob, G.extract_params(N, 1, precision=G.GRAVER_FP32, init_mode=1, collect=0,
                                                  form=G.GRAVER_FORM_SPARSE), state=st)
        assert torch.equal(st["z"], _dev(z0))
        return
    for t_teacher in (0, 25):
        z, mm, vv, _ = S.descend(B, z0, t_teacher, P_) if t_teacher else (z0, np.zeros_like(z0), np.zeros_like(z0), 0)
        zo, mo, _, _ = S.descend(B, z, 1, P_, m0=mm, v0=vv, t0=t_teacher)
        prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
        st = {"z": _dev(z), "m": _dev(mm), "v": _dev(vv)}
        precision = G.GRAVER_BF16 if prec == "bf16" else G.GRAVER_FP32
        form = G.GRAVER_FORM_SPARSE if prec == "fp32-sparse" else G.GRAVER_FORM_DENSE
        prm = G.extract_params(N, 1, precision=precision, init_mode=1, t0=t_teacher, collect=0, form=form)
        G.extract(ctx, prob, prm, state=st)
        err, flagged = _check_step(B, z, mm, vv, t_teacher + 1, st["z"].cpu().numpy(), zo)
        _say("big teacher-forced", n, prec, t_teacher, "max err", float(err.max()), "kink starts", flagged)
        assert np.median(_relerr(st["m"].cpu().numpy(), mo)) <= TOL


@pytest.mark.parametrize("shape", SHAPES, ids=[f"n{n}" for n, _ in SHAPES])
def test_big_short_horizon_and_sets(G, ctx, shape):
    """20 binary32 steps match the oracle; the binary32 set equals the
    binary64 GPU set of the same starts up to rounding-edge cases, and every
    key is verified."""
    n, m = shape
    inst, B, _ = _inst(n, m)
    _say("big short horizon", n, B.shape[1])
    N = 512
    z0 = W.gaussian_starts(N, B.shape[1], 2.0, 78)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    st = {"z": _dev(z0)}
    G.extract(ctx, prob, G.extract_params(N, 20, precision=G.GRAVER_FP32, form=G.GRAVER_FORM_DENSE, init_mode=1, collect=0), state=st)
    zo, _, _, _ = S.descend(B, z0, 20, P_)
    err = _relerr(st["z"].cpu().numpy(), zo)
    _say("big short horizon", n, "within tol", float(np.mean(err <= TOL)), "max", float(err.max()))
    assert np.mean(err <= TOL) >= 0.95
    # starts near the origin: after 60 steps most rounded iterates map into
    # the box (sigma 2 starts need thousands of steps before they do)
    z1 = W.gaussian_starts(N, B.shape[1], 0.3, 78)
    k32, s32 = G.extract(ctx, prob, G.extract_params(N, 60, precision=G.GRAVER_FP32, form=G.GRAVER_FORM_DENSE, init_mode=1,
                                                        pool_capacity=1 << 20), state={"z": _dev(z1)})
    k64, s64 = G.extract(ctx, prob, G.extract_params(N, 60, precision=G.GRAVER_FP64, init_mode=1,
                                                        pool_capacity=1 << 20), state={"z": _dev(z1)})
    a = {tuple(r) for r in k32.cpu().numpy().tolist()}
    b = {tuple(r) for r in k64.cpu().numpy().tolist()}
    jac = len(a & b) / max(1, len(a | b))
    _say("big sets", n, "fp32", len(a), "fp64", len(b), "jaccard", jac, "events", s32["inbox_events"], s64["inbox_events"])
    assert len(b) > 0 and jac >= 0.9
    K = k32.cpu().numpy().astype(np.int64)
    assert np.all(K @ inst.A.T == 0) and np.all(np.abs(K) <= (inst.u - inst.l)[None, :])
    assert s32["out_of_range"] == 0


def test_big_fp64_sets_equal_oracle(G, ctx):
    """The binary64 path at n = 200 returns exactly the oracle's set."""
    inst, B, _ = _inst(200, 40)
    _say("big fp64 vs oracle")
    N, T = 64, 60
    z0 = W.gaussian_starts(N, B.shape[1], 0.3, 81)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    st = {"z": _dev(z0)}
    k64, _ = G.extract(ctx, prob, G.extract_params(N, T, precision=G.GRAVER_FP64, init_mode=1,
                                                    pool_capacity=1 << 18), state=st)
    keys, (zo, _, _) = S.extract(inst.A, B, inst.l, inst.u, z0, T, P_)
    assert np.array_equal(st["z"].cpu().numpy().view(np.uint64), zo.view(np.uint64))
    got = sorted(tuple(r) for r in k64.cpu().numpy().astype(np.int64).tolist())
    assert got == [tuple(k) for k in keys]
    _say("big fp64 vs oracle", "keys", len(got))


def test_big_resume_and_overflow_replay(G, ctx):
    """Chunked calls reproduce one long call bit for bit, and a small pool
    capacity (log overflow, replay) gives the same set."""
    inst, B, _ = _inst(200, 40)
    _say("big resume / replay")
    N = 1024
    z0 = W.gaussian_starts(N, B.shape[1], 0.3, 79)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    zero = lambda: torch.zeros((N, B.shape[1]), dtype=torch.float64, device="cuda")
    st1 = {"z": _dev(z0), "m": zero(), "v": zero()}
    G.extract(ctx, prob, G.extract_params(N, 30, precision=G.GRAVER_FP32, form=G.GRAVER_FORM_DENSE, init_mode=1, collect=0), state=st1)
    G.extract(ctx, prob, G.extract_params(N, 20, precision=G.GRAVER_FP32, form=G.GRAVER_FORM_DENSE, init_mode=1, t0=30, collect=0), state=st1)
    st2 = {"z": _dev(z0), "m": zero(), "v": zero()}
    G.extract(ctx, prob, G.extract_params(N, 50, precision=G.GRAVER_FP32, form=G.GRAVER_FORM_DENSE, init_mode=1, collect=0), state=st2)
    assert torch.equal(st1["z"], st2["z"]) and torch.equal(st1["m"], st2["m"])
    big = G.extract_params(N, 80, precision=G.GRAVER_FP32, form=G.GRAVER_FORM_DENSE, init_mode=1, pool_capacity=1 << 20)
    kb, sb = G.extract(ctx, prob, big, state={"z": _dev(z0)})
    cap = max(64, int(kb.shape[0] * 1.02))
    if sb["inbox_events"] > cap:
        ks, _ = G.extract(ctx, prob, G.extract_params(N, 80, precision=G.GRAVER_FP32, form=G.GRAVER_FORM_DENSE, init_mode=1,
                                                       pool_capacity=cap), state={"z": _dev(z0)})
        assert torch.equal(kb, ks)
    _say("big resume / replay", "unique", kb.shape[0], "events", sb["inbox_events"])

"""GPU parity of the matrix-core descent for wide bases (d > 256), whose
coordinates are split over 2 or 4 waves per start group: the workload with
m=50, n=400 (d=350, sparse A, quartic objective) and identity-block
instances with n=800 (d=640) and n=1000 (d=800), against the binary64
oracle and the binary64 GPU path."""
import numpy as np
import pytest

from oracle import lattice
from oracle import surrogate as S
from paper_2412_13576_amd import workloads as W
from tests.test_gpu_fp32 import TOL, _check_step, _relerr

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
P_ = S.AdamParams()

# (name, builder, LLL) -- the identity-block bases are taken without LLL
# (B = [-C; I] is already short; exact LLL at d = 800 takes minutes)
CASES = [
    ("quartic_n400_d350", lambda: W.quartic_instance(), True),
    ("idblock_n800_d640", lambda: W.identity_block_instance(5800, 800, 160), False),
    ("idblock_n1000_d800", lambda: W.identity_block_instance(6000, 1000, 200), False),
]
IDS = [c[0] for c in CASES]


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


def _inst(name):
    if name not in _cache:
        _, build, lll = CASES[IDS.index(name)]
        inst = build()
        _cache[name] = (inst, lattice.kernel_basis(inst.A, lll=lll))
    return _cache[name]


def _pf(G, prec):
    """(precision, form) of a case name: binary32 in the form the library
    picks (the sparse form on the quartic basis), binary32 on matrix cores,
    or bf16 on matrix cores."""
    return {"fp32": (G.GRAVER_FP32, G.GRAVER_FORM_AUTO), "fp32-dense": (G.GRAVER_FP32, G.GRAVER_FORM_DENSE),
            "bf16": (G.GRAVER_BF16, G.GRAVER_FORM_AUTO)}[prec]


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name", IDS)
@pytest.mark.parametrize("prec", ["fp32", "fp32-dense", "bf16"])
def test_wide_teacher_forced_single_step(G, ctx, name, prec):
    inst, B = _inst(name)
    _say("wide teacher-forced", name, prec)
    N = 50                      # ragged: the last start group holds 2 starts
    z0 = W.gaussian_starts(N, B.shape[1], 2.0, 77)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    precision, form = _pf(G, prec)
    for t_teacher in (0, 25):
        z, mm, vv, _ = (S.descend(B, z0, t_teacher, P_) if t_teacher
                        else (z0, np.zeros_like(z0), np.zeros_like(z0), 0))
        zo, mo, _, _ = S.descend(B, z, 1, P_, m0=mm, v0=vv, t0=t_teacher)
        st = {"z": _dev(z), "m": _dev(mm), "v": _dev(vv)}
        G.extract(ctx, prob, G.extract_params(N, 1, precision=precision, init_mode=1, t0=t_teacher, collect=0,
                                              form=form), state=st)
        err, flagged = _check_step(B, z, mm, vv, t_teacher + 1, st["z"].cpu().numpy(), zo)
        _say("wide teacher-forced", name, prec, t_teacher, "max err", float(err.max()), "kink starts", flagged)
        assert np.median(_relerr(st["m"].cpu().numpy(), mo)) <= TOL


@pytest.mark.parametrize("name", IDS)
def test_wide_short_horizon_and_sets(G, ctx, name):
    """20 binary32 steps match the oracle; the binary32 and bf16 sets equal
    the binary64 GPU set of the same starts up to rounding-edge cases, and
    every key is verified."""
    inst, B = _inst(name)
    _say("wide short horizon", name)
    N = 512
    z0 = W.gaussian_starts(N, B.shape[1], 2.0, 78)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    st = {"z": _dev(z0)}
    G.extract(ctx, prob, G.extract_params(N, 20, precision=G.GRAVER_FP32, init_mode=1, collect=0), state=st)
    zo, _, _, _ = S.descend(B, z0, 20, P_)
    err = _relerr(st["z"].cpu().numpy(), zo)
    _say("wide short horizon", name, "within tol", float(np.mean(err <= TOL)), "max", float(err.max()))
    assert np.mean(err <= TOL) >= 0.95
    z1 = W.gaussian_starts(N, B.shape[1], 0.3, 78)
    sets = {}
    for prec in ("fp64", "fp32", "bf16"):
        precision = {"fp64": G.GRAVER_FP64, "fp32": G.GRAVER_FP32, "bf16": G.GRAVER_BF16}[prec]
        k, s = G.extract(ctx, prob, G.extract_params(N, 60, precision=precision, init_mode=1,
                                                      pool_capacity=1 << 20), state={"z": _dev(z1)})
        sets[prec] = {tuple(r) for r in k.cpu().numpy().tolist()}
        if prec != "fp64":
            K = k.cpu().numpy().astype(np.int64)
            assert np.all(K @ inst.A.T == 0) and np.all(np.abs(K) <= (inst.u - inst.l)[None, :])
            assert s["out_of_range"] == 0
    for prec in ("fp32", "bf16"):
        a, b = sets[prec], sets["fp64"]
        jac = len(a & b) / max(1, len(a | b))
        _say("wide sets", name, prec, len(a), "fp64", len(b), "jaccard", jac)
        assert len(b) > 0 and jac >= 0.9


def test_wide_fp64_sets_equal_oracle(G, ctx):
    """The binary64 path at n = 400, d = 350 returns exactly the oracle's set
    and final iterates."""
    inst, B = _inst("quartic_n400_d350")
    _say("wide fp64 vs oracle")
    N, T = 32, 40
    z0 = W.gaussian_starts(N, B.shape[1], 0.3, 81)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    st = {"z": _dev(z0)}
    k64, _ = G.extract(ctx, prob, G.extract_params(N, T, precision=G.GRAVER_FP64, init_mode=1,
                                                    pool_capacity=1 << 18), state=st)
    keys, (zo, _, _) = S.extract(inst.A, B, inst.l, inst.u, z0, T, P_)
    assert np.array_equal(st["z"].cpu().numpy().view(np.uint64), zo.view(np.uint64))
    got = sorted(tuple(r) for r in k64.cpu().numpy().astype(np.int64).tolist())
    assert got == [tuple(k) for k in keys]
    _say("wide fp64 vs oracle", "keys", len(got))


@pytest.mark.parametrize("prec", ["fp32", "fp32-dense", "bf16"])
def test_wide_resume_and_overflow_replay(G, ctx, prec):
    """Chunked calls reproduce one long call bit for bit (the bf16 form is
    resumed inside its bf16 phase), and a small pool capacity (log
    overflow, replay) gives the same set."""
    inst, B = _inst("quartic_n400_d350")
    _say("wide resume / replay", prec)
    N = 1000
    precision, form = _pf(G, prec)
    z0 = W.gaussian_starts(N, B.shape[1], 0.3, 79)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    zero = lambda: torch.zeros((N, B.shape[1]), dtype=torch.float64, device="cuda")
    st1 = {"z": _dev(z0), "m": zero(), "v": zero()}
    G.extract(ctx, prob, G.extract_params(N, 30, precision=precision, init_mode=1, collect=0, form=form), state=st1)
    G.extract(ctx, prob, G.extract_params(N, 20, precision=precision, init_mode=1, t0=30, collect=0, form=form),
              state=st1)
    st2 = {"z": _dev(z0), "m": zero(), "v": zero()}
    G.extract(ctx, prob, G.extract_params(N, 50, precision=precision, init_mode=1, collect=0, form=form), state=st2)
    assert torch.equal(st1["z"], st2["z"]) and torch.equal(st1["m"], st2["m"])
    big = G.extract_params(N, 80, precision=precision, init_mode=1, pool_capacity=1 << 20, form=form)
    kb, sb = G.extract(ctx, prob, big, state={"z": _dev(z0)})
    cap = kb.shape[0]           # every distinct key fits; the events do not
    assert sb["inbox_events"] > cap
    ks, _ = G.extract(ctx, prob, G.extract_params(N, 80, precision=precision, init_mode=1, pool_capacity=cap,
                                                  form=form), state={"z": _dev(z0)})
    assert torch.equal(kb, ks)
    _say("wide resume / replay", prec, "unique", kb.shape[0], "events", sb["inbox_events"], "row entries",
         sb["row_entries"])
    assert (sb["row_entries"] > 0) == (prec == "fp32")


def test_quartic_precision_forms_equal_recall(G, ctx):
    """The precision comparison on the quartic workload (n = 400, d = 350):
    binary32 vs bf16 (last 10% of the steps polished in binary32) from the
    same 8192 box starts x 2000 steps; each form's recall against the
    filtered union of both sets.  Equal recall means the bf16 form is within
    0.01 of the binary32 form."""
    inst, B = _inst("quartic_n400_d350")
    P = lattice.coordinate_projector(B)
    N, T = 8192, 2000
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    sets, times = {}, {}
    for name, prec, pol in (("fp32", G.GRAVER_FP32, 0), ("bf16", G.GRAVER_BF16, T // 10)):
        _say("quartic recall", name)
        prm = G.extract_params(N, T, precision=prec, init_mode=0, seed=77, polish_iters=pol, pool_capacity=1 << 23,
                               any_order=True)
        k, st = G.extract(ctx, prob, prm)
        sets[name] = G.filter_minimal(ctx, k)
        times[name] = st["ms_descent"]
        del k
    ref = G.filter_minimal(ctx, torch.cat([sets["fp32"], sets["bf16"]]))
    rv = np.ascontiguousarray(ref.cpu().numpy()).view(np.dtype((np.void, ref.shape[1]))).ravel()
    rec = {}
    for name, F in sets.items():
        fv = np.ascontiguousarray(F.cpu().numpy()).view(np.dtype((np.void, F.shape[1]))).ravel()
        rec[name] = float(np.isin(rv, fv).sum() / max(1, rv.size))
    _say("quartic recall", rec, "descent ms", times)
    assert rec["bf16"] >= rec["fp32"] - 0.01

"""The integer stages of the matrix-core extraction against an exact host
computation from the GPU's own iterates (Algorithm 2: every iterate z^t,
t = 1..T, is rounded to r^t and g = B r^t is collected when nonzero and
inside [l - u, u - l]).

A T-step launch is chained as T one-step launches whose state is read back
after each step (resumption is bit-exact, so these are the same iterates);
the host rounds each iterate (ties to even) and forms B r exactly, and the
distinct in-box nonzero results must be exactly the key set of one T-step
launch with collection.  This covers the incremental g += B (r - r_prev) of
the small-basis kernel and the one-iteration-late B r of the large-basis
kernel at the benchmark's launch shapes (box starts, uniform box), in
binary32 and bf16.  Iterates beyond a kernel's exact range yield no
candidate in that kernel; the host applies the same rule, and the split
test checks that the set does not depend on how a run is split."""
import numpy as np
import pytest

from oracle import lattice
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


_BASES = {}


def _basis(kind):
    if kind not in _BASES:
        inst = W.qp_instance(2000) if kind == "qp" else W.quartic_instance(3000)
        B = lattice.kernel_basis(inst.A)
        _BASES[kind] = (inst, B, lattice.coordinate_projector(B))
    return _BASES[kind]


def _void(a):
    a = np.ascontiguousarray(a, dtype=np.int8)
    return a.view(np.dtype((np.void, a.shape[1]))).ravel()


class _HostSet:
    """Distinct in-box nonzero B r over the iterates fed to add()."""

    def __init__(self, B, l, u, rlim):
        self.Bt = B.T.astype(np.float64)
        self.lim = (u - l).astype(np.float64)
        self.rlim = rlim
        self.parts = []
        self.r_prev = None
        self.events = 0  # changed, in range, nonzero, in the box

    def add(self, z):
        r = np.rint(z)
        inr = np.all(np.abs(r) <= self.rlim, axis=1)
        changed = np.ones(r.shape[0], bool) if self.r_prev is None else np.any(r != self.r_prev, axis=1)
        self.r_prev = r
        g = r[inr] @ self.Bt  # exact: every partial sum is an integer far below 2^53
        ok = np.all(np.abs(g) <= self.lim, axis=1) & np.any(g != 0, axis=1)
        self.events += int((ok & changed[inr]).sum())
        if ok.any():
            self.parts.append(np.unique(_void(g[ok].astype(np.int8))))

    def keys(self):
        return np.unique(np.concatenate(self.parts)) if self.parts else np.zeros(0, np.dtype((np.void, 1)))


def _chain(G, ctx, prob, N, d, T, prec, seed, z0=None, lr=0.003, form=0):
    """T one-step launches from box starts (or z0); yields z^1..z^T."""
    dev = "cuda"
    st = {"z": torch.empty((N, d), dtype=torch.float64, device=dev) if z0 is None else z0.clone(),
          "m": torch.zeros((N, d), dtype=torch.float64, device=dev),
          "v": torch.zeros((N, d), dtype=torch.float64, device=dev)}
    for t in range(T):
        init = 0 if (t == 0 and z0 is None) else 1
        prm = G.extract_params(N, 1, precision=prec, init_mode=init, seed=seed, t0=t, collect=0, lr=lr,
                               pool_capacity=1, form=form)
        G.extract(ctx, prob, prm, state=st)
        yield st["z"].cpu().numpy()


def _single(G, ctx, prob, N, d, T, prec, seed, z0=None, lr=0.003, cap=1 << 22, form=0):
    st = None
    if z0 is not None:
        st = {"z": z0.clone()}
    prm = G.extract_params(N, T, precision=prec, init_mode=0 if z0 is None else 1, seed=seed,
                           pool_capacity=cap, lr=lr, form=form)
    keys, stats = G.extract(ctx, prob, prm, state=st)
    return keys.cpu().numpy(), stats


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_small_kernel_candidates_exact_at_benchmark_launch(G, ctx, prec):
    """QP workload (n = 100, d = 80, uniform box [-10, 10]), 65536 box starts,
    40 iterations: the small-basis kernel's keys are exactly the host set."""
    inst, B, P = _basis("qp")
    n, d = B.shape
    N, T = 65536, 40
    pv = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    rlim = float(np.floor(2.0 ** 24 / np.abs(B).sum(axis=1).max()))
    hs = _HostSet(B, inst.l, inst.u, rlim)
    _say("small kernel chain", prec)
    for z in _chain(G, ctx, prob, N, d, T, pv, seed=11):
        hs.add(z)
    keys, stats = _single(G, ctx, prob, N, d, T, pv, seed=11)
    _say("small kernel", prec, "keys", keys.shape[0], "host", hs.keys().size)
    assert stats["out_of_range"] == 0
    assert stats["inbox_events"] == hs.events
    assert np.array_equal(np.unique(_void(keys)), hs.keys())
    assert keys.shape[0] > 10000


@pytest.mark.parametrize("prec,form", [("fp32", "dense"), ("bf16", "dense"), ("fp32", "sparse")])
def test_large_kernel_candidates_exact(G, ctx, prec, form):
    """Quartic workload (n = 400, d = 350), 8192 box starts, 40 iterations:
    the large matrix-core kernel (coordinates of a start split over waves,
    exact range |r| <= 256) and the sparse form (one start per wavefront,
    exact range floor(2^24 / max row l1 of B); the form binary32 calls take
    on this basis)."""
    inst, B, P = _basis("quartic")
    n, d = B.shape
    N, T = 8192, 40
    pv = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
    fm = G.GRAVER_FORM_DENSE if form == "dense" else G.GRAVER_FORM_SPARSE
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    rlim = 256.0 if form == "dense" else float(np.floor(2.0 ** 24 / np.abs(B).sum(axis=1).max()))
    hs = _HostSet(B, inst.l, inst.u, rlim)
    _say("large kernel chain", prec, form)
    for z in _chain(G, ctx, prob, N, d, T, pv, seed=12, form=fm):
        hs.add(z)
    keys, stats = _single(G, ctx, prob, N, d, T, pv, seed=12, form=fm)
    _say("large kernel", prec, form, "keys", keys.shape[0], "host", hs.keys().size)
    if form == "sparse":
        assert stats["row_entries"] > 0 and stats["tile_slices"] == 0
    else:
        assert stats["row_entries"] == 0 and stats["tile_slices"] > 0
    assert stats["out_of_range"] == 0
    assert stats["inbox_events"] == hs.events
    assert np.array_equal(np.unique(_void(keys)), hs.keys())
    assert keys.shape[0] > 1000


def test_large_kernel_out_of_range_iterates(G, ctx):
    """Starts with a coordinate near the large kernel's exact range |r| <= 256
    and a large step, so iterates leave and re-enter it: each out-of-range
    iterate is skipped alone, the set equals the host set, and a run split
    into three launches returns the same set and count."""
    inst, B, P = _basis("quartic")
    n, d = B.shape
    N, T, lr = 512, 60, 0.2
    rng = np.random.default_rng(31)
    z0 = rng.standard_normal((N, d)) * 0.5
    z0[: N // 2, 0] = 256.0 + rng.uniform(-1.5, 1.5, N // 2)
    z0d = torch.tensor(z0, device="cuda")
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    hs = _HostSet(B, inst.l, inst.u, 256.0)
    dense = G.GRAVER_FORM_DENSE
    for z in _chain(G, ctx, prob, N, d, T, G.GRAVER_FP32, seed=0, z0=z0d, lr=lr, form=dense):
        hs.add(z)
    keys, stats = _single(G, ctx, prob, N, d, T, G.GRAVER_FP32, seed=0, z0=z0d, lr=lr, form=dense)
    _say("out of range", stats["out_of_range"], "keys", keys.shape[0])
    assert stats["out_of_range"] > 0
    assert np.array_equal(np.unique(_void(keys)), hs.keys())
    # the same run in three launches
    st = {"z": z0d.clone(), "m": torch.zeros_like(z0d), "v": torch.zeros_like(z0d)}
    parts, oor = [], 0
    for k in range(3):
        prm = G.extract_params(N, T // 3, precision=G.GRAVER_FP32, init_mode=1, t0=k * (T // 3),
                               pool_capacity=1 << 20, lr=lr, form=dense)
        kk, s = G.extract(ctx, prob, prm, state=st)
        parts.append(_void(kk.cpu().numpy()))
        oor += s["out_of_range"]
    assert np.array_equal(np.unique(np.concatenate(parts)), hs.keys())
    # a launch's first iterate counts as changed, so the split run may count
    # a few more out-of-range iterates than the single run
    assert oor >= stats["out_of_range"]


def test_small_kernel_out_of_range_split(G, ctx):
    """Small-basis kernel with starts straddling its exact range
    floor(2^24 / max row l1 of B) and a step of about one unit: out-of-range
    iterates are skipped alone, the set equals the host set, and a split run
    returns the same set and count."""
    inst, B, P = _basis("qp")
    n, d = B.shape
    rlim = float(np.floor(2.0 ** 24 / np.abs(B).sum(axis=1).max()))
    N, T, lr = 1024, 30, 1.0
    rng = np.random.default_rng(32)
    z0 = rng.standard_normal((N, d)) * 0.5
    z0[: N // 2, 3] = rlim + rng.uniform(-2.5, 2.5, N // 2)
    z0d = torch.tensor(z0, device="cuda")
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    hs = _HostSet(B, inst.l, inst.u, rlim)
    for z in _chain(G, ctx, prob, N, d, T, G.GRAVER_FP32, seed=0, z0=z0d, lr=lr):
        hs.add(z)
    keys, stats = _single(G, ctx, prob, N, d, T, G.GRAVER_FP32, seed=0, z0=z0d, lr=lr)
    _say("small out of range", stats["out_of_range"], "keys", keys.shape[0])
    assert stats["out_of_range"] > 0
    assert np.array_equal(np.unique(_void(keys)), hs.keys())
    st = {"z": z0d.clone(), "m": torch.zeros_like(z0d), "v": torch.zeros_like(z0d)}
    parts, oor = [], 0
    for k in range(3):
        prm = G.extract_params(N, T // 3, precision=G.GRAVER_FP32, init_mode=1, t0=k * (T // 3),
                               pool_capacity=1 << 20, lr=lr)
        kk, s = G.extract(ctx, prob, prm, state=st)
        parts.append(_void(kk.cpu().numpy()))
        oor += s["out_of_range"]
    assert np.array_equal(np.unique(np.concatenate(parts)), hs.keys())
    # a launch's first iterate counts as changed, so the split run may count
    # a few more out-of-range iterates than the single run
    assert oor >= stats["out_of_range"]


@pytest.mark.parametrize("kind", ["quartic", "qp"])
def test_sparse_form_out_of_range_split(G, ctx, kind):
    """Sparse form with starts straddling its exact range floor(2^24 / max row
    l1 of B) and a step of about one unit: out-of-range iterates are skipped
    alone, the set equals the host set, and a run split into three launches
    returns the same set (on the quartic basis, and on the QP basis, where the
    form is asked for explicitly: the small matrix-core kernel would run)."""
    inst, B, P = _basis(kind)
    n, d = B.shape
    rlim = float(np.floor(2.0 ** 24 / np.abs(B).sum(axis=1).max()))
    N, T, lr = 1000, 30, 1.0           # ragged: 1000 starts = 62 groups of 16 + 8
    rng = np.random.default_rng(33)
    z0 = rng.standard_normal((N, d)) * 0.5
    z0[: N // 2, 3] = rlim + rng.uniform(-2.5, 2.5, N // 2)
    z0d = torch.tensor(z0, device="cuda")
    sp = G.GRAVER_FORM_SPARSE
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    hs = _HostSet(B, inst.l, inst.u, rlim)
    for z in _chain(G, ctx, prob, N, d, T, G.GRAVER_FP32, seed=0, z0=z0d, lr=lr, form=sp):
        hs.add(z)
    keys, stats = _single(G, ctx, prob, N, d, T, G.GRAVER_FP32, seed=0, z0=z0d, lr=lr, form=sp)
    _say("sparse out of range", kind, stats["out_of_range"], "keys", keys.shape[0], "entries", stats["row_entries"])
    assert stats["row_entries"] > 0
    assert stats["out_of_range"] > 0
    assert stats["inbox_events"] == hs.events
    assert np.array_equal(np.unique(_void(keys)), hs.keys())
    st = {"z": z0d.clone(), "m": torch.zeros_like(z0d), "v": torch.zeros_like(z0d)}
    parts, oor = [], 0
    for k in range(3):
        prm = G.extract_params(N, T // 3, precision=G.GRAVER_FP32, init_mode=1, t0=k * (T // 3),
                               pool_capacity=1 << 20, lr=lr, form=sp)
        kk, s = G.extract(ctx, prob, prm, state=st)
        parts.append(_void(kk.cpu().numpy()))
        oor += s["out_of_range"]
    assert np.array_equal(np.unique(np.concatenate(parts)), hs.keys())
    assert oor >= stats["out_of_range"]

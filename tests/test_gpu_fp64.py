"""GPU parity of the binary64 path against the oracle: extraction (sets and
iterates), start generation, filter and augmentation, all through the C ABI."""
import numpy as np
import pytest

from oracle import lattice, philox
from oracle import surrogate as S
from oracle.augment import Objective, augment as o_augment
from oracle.conformal import canonical
from oracle.minimal import filter_minimal as o_filter
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


def _rows(t):
    return [tuple(int(v) for v in r) for r in t.cpu().numpy()]


def _dev(x, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")


@pytest.mark.parametrize("seed", [1000, 1001, 1002, 1003, 1004])
def test_tiny_extraction_bit_exact(G, ctx, seed):
    """Tiny instance, 1024 starts z0 ~ N(0, 4I), 500 binary64 steps: the
    extracted set and the final iterates equal the oracle's bit for bit."""
    _say("tiny extraction", seed)
    inst = W.tiny_instance(seed)
    B = lattice.kernel_basis(inst.A)
    z0 = W.gaussian_starts(1024, B.shape[1], 2.0, seed + 1)
    keys_o, (zo, mo, vo) = S.extract(inst.A, B, inst.l, inst.u, z0, 500, S.AdamParams())
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    st = {"z": _dev(z0), "m": torch.zeros_like(_dev(z0)), "v": torch.zeros_like(_dev(z0))}
    prm = G.extract_params(1024, 500, precision=G.GRAVER_FP64, init_mode=1, pool_capacity=1 << 18)
    keys, stats = G.extract(ctx, prob, prm, state=st)
    assert _rows(keys) == keys_o
    assert stats["verified"] == len(keys_o) and stats["out_of_range"] == 0
    assert np.array_equal(st["z"].cpu().numpy(), zo)
    assert np.array_equal(st["m"].cpu().numpy(), mo)
    assert np.array_equal(st["v"].cpu().numpy(), vo)
    # recall against the brute-force Graver basis in [-6, 6]^8
    from tests.golden_io import tiny_graver_box6
    Gb = tiny_graver_box6()[seed]
    rec = len(Gb & set(keys_o)) / len(Gb)
    _say("recall vs brute force", seed, round(rec, 3), "unique", len(keys_o))


def test_tiny_trajectory_checkpoints(G, ctx):
    """Iterates at t = 1, 10, 100, 500 through chunked (resumed) calls are
    within 1e-9 relative of the oracle (and in fact identical)."""
    _say("trajectory checkpoints")
    inst = W.tiny_instance(1002)
    B = lattice.kernel_basis(inst.A)
    z0 = W.gaussian_starts(512, B.shape[1], 2.0, 77)
    p = S.AdamParams()
    _, _, _, snaps = S.descend(B, z0, 500, p, record=(1, 10, 100, 500))
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    st = {"z": _dev(z0), "m": torch.zeros_like(_dev(z0)), "v": torch.zeros_like(_dev(z0))}
    t = 0
    for tt in (1, 10, 100, 500):
        prm = G.extract_params(512, tt - t, precision=G.GRAVER_FP64, init_mode=1, t0=t, collect=0)
        G.extract(ctx, prob, prm, state=st)
        t = tt
        zg = st["z"].cpu().numpy()
        zr = snaps[tt]
        err = np.abs(zg - zr).max(axis=1) / np.maximum(np.abs(zr).max(axis=1), 1.0)
        assert err.max() <= 1e-9
        assert np.array_equal(zg, zr)


def test_philox_starts_bit_exact(G, ctx):
    """init_mode 0: g ~ U(l-u, u-l) by Philox4x32-10 and z0 = P g equal the
    oracle's draws exactly (P injected)."""
    _say("philox starts")
    inst = W.tiny_instance(1001)
    B = lattice.kernel_basis(inst.A)
    P = lattice.coordinate_projector(B)
    N = 3000
    _, zo = philox.box_starts(P, inst.l, inst.u, N, seed=0x1234567890ABCDEF, first_start=17)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    st = {"z": torch.zeros((N, B.shape[1]), dtype=torch.float64, device="cuda")}
    prm = G.extract_params(N, 0, precision=G.GRAVER_FP64, init_mode=0, seed=0x1234567890ABCDEF,
                           first_start=17, collect=0)
    G.extract(ctx, prob, prm, state=st)
    assert np.array_equal(st["z"].cpu().numpy(), zo)


def test_extraction_deterministic_and_resume(G, ctx):
    """Two identical calls give identical sets; 30 + 50 resumed steps give
    the union of the two chunks' oracle sets."""
    _say("determinism / resume")
    inst = W.tiny_instance(1003)
    B = lattice.kernel_basis(inst.A)
    z0 = W.gaussian_starts(2048, B.shape[1], 2.0, 9)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    prm = G.extract_params(2048, 80, precision=G.GRAVER_FP64, init_mode=1, pool_capacity=1 << 16)
    k1, _ = G.extract(ctx, prob, prm, state={"z": _dev(z0)})
    k2, _ = G.extract(ctx, prob, prm, state={"z": _dev(z0)})
    assert torch.equal(k1, k2)
    ko, (z30, m30, v30) = S.extract(inst.A, B, inst.l, inst.u, z0, 30, S.AdamParams())
    ko2, _ = S.extract(inst.A, B, inst.l, inst.u, z30, 50, S.AdamParams(), m0=m30, v0=v30, t0=30)
    st = {"z": _dev(z30), "m": _dev(m30), "v": _dev(v30)}
    prm2 = G.extract_params(2048, 50, precision=G.GRAVER_FP64, init_mode=1, t0=30, pool_capacity=1 << 16)
    k3, _ = G.extract(ctx, prob, prm2, state=st)
    assert _rows(k3) == ko2
    assert sorted(set(_rows(k1))) == sorted(set(ko) | set(ko2))


def test_extraction_error_paths(G, ctx):
    _say("extract errors")
    inst = W.tiny_instance(1000)
    B = lattice.kernel_basis(inst.A)
    z0 = W.gaussian_starts(256, B.shape[1], 2.0, 3)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B)
    prm = G.extract_params(256, 200, precision=G.GRAVER_FP64, init_mode=1, pool_capacity=4)
    with pytest.raises(G.GraverError) as e:
        G.extract(ctx, prob, prm, state={"z": _dev(z0)})
    assert e.value.status == -5
    prm = G.extract_params(256, 200, precision=G.GRAVER_FP64, init_mode=1, pool_capacity=1 << 14)
    with pytest.raises(G.GraverError) as e:
        G.extract(ctx, prob, prm, state={"z": _dev(z0)}, keys_cap=2)
    assert e.value.status == -8
    Bbad = B.copy()
    Bbad[0, 0] += 1
    bad = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, Bbad)
    with pytest.raises(G.GraverError) as e:
        G.extract(ctx, bad, prm, state={"z": _dev(z0)})
    assert e.value.status == -3
    wide = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l - 100, inst.u + 100, B)
    with pytest.raises(G.GraverError) as e:
        G.extract(ctx, wide, prm, state={"z": _dev(z0)})
    assert e.value.status == -1
    # empty result (T = 0 collects nothing) is not an error
    prm0 = G.extract_params(256, 0, precision=G.GRAVER_FP64, init_mode=1, pool_capacity=16)
    k, _ = G.extract(ctx, prob, prm0, state={"z": _dev(z0)})
    assert k.shape[0] == 0


def _filter_cases():
    rng = np.random.default_rng(4)
    cases = []
    inst = W.tiny_instance(1001)
    B = lattice.kernel_basis(inst.A)
    z0 = W.gaussian_starts(1024, B.shape[1], 2.0, 5)
    keys, _ = S.extract(inst.A, B, inst.l, inst.u, z0, 300, S.AdamParams())
    cases.append(("tiny-extracted", np.array(keys, dtype=np.int8)))
    flip = np.array([k if rng.random() < 0.5 else tuple(-x for x in k) for k in keys], dtype=np.int8)
    cases.append(("tiny-flipped-dup", np.concatenate([flip, flip[:50], np.zeros((3, 8), np.int8)])))
    for n, K in [(13, 700), (70, 3000), (130, 1500)]:
        X = rng.integers(-2, 3, size=(K, n)) * (rng.random((K, n)) < 0.15)
        X[::7] = X[::7] * 2
        cases.append((f"random-n{n}", X.astype(np.int8)))
    cases.append(("single", np.array([[0, -3, 1]], dtype=np.int8)))
    # dense keys (the shape the QP workload produces) and a structured set in
    # which many keys have witnesses: both exercise the sign-pattern index
    D = rng.integers(-12, 13, size=(2500, 100))
    D[rng.random(D.shape) < 0.09] = 0
    cases.append(("dense-n100", D.astype(np.int8)))
    base = rng.integers(-2, 3, size=(600, 20)) * (rng.random((600, 20)) < 0.4)
    mult = base[rng.integers(0, 600, size=3000)] + base[rng.integers(0, 600, size=3000)]
    cases.append(("sums-n20", np.concatenate([base, mult]).astype(np.int8)))
    return cases


@pytest.mark.parametrize("name,X", _filter_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_filter_bit_exact(G, ctx, name, X):
    _say("filter", name, X.shape)
    want = o_filter([tuple(int(v) for v in r) for r in X])
    got = G.filter_minimal(ctx, torch.tensor(X, device="cuda"))
    assert _rows(got) == want


@pytest.mark.parametrize("shape", ["sparse-600k", "dense-one-pattern-60k"])
def test_filter_closed_form_large(G, ctx, shape):
    """Large key sets whose minimal elements are known: atoms on distinct
    supports of one size plus sums of sign-compatible atom pairs; the filter
    must return exactly the atoms.  The sparse set spreads over the widest
    sign-pattern index; the dense nonnegative set puts nearly every key in
    one bucket, which the join splits into many chunks."""
    if shape == "sparse-600k":
        X, atoms = W.antichain_with_sums(n=100, n_atoms=3000, support=6, n_sums=600_000, seed=8)
    else:
        X, atoms = W.antichain_with_sums(n=100, n_atoms=2000, support=90, n_sums=60_000, seed=9,
                                         positive=True)
    _say("filter closed form", shape, X.shape)
    want = sorted({canonical(a) for a in atoms})
    got = G.filter_minimal(ctx, torch.tensor(X, device="cuda"))
    assert got.shape[0] == len(want)
    assert _rows(got) == want


def _profile_set(n=100, n_atoms=24000, support=60, n_prof=16, n_sums=2_500_000, mag=60, seed=10):
    """Closed-form key set of about 2.35 M distinct keys with entries up to
    +-120: atoms with distinct supports of one size (an antichain) whose
    signs follow one of n_prof sign profiles, plus sums of two atoms of the
    same profile (each lies above both summands).  The minimal elements are
    exactly the atoms."""
    rng = np.random.default_rng(seed)
    prof = rng.choice(np.array([-1, 1], np.int16), size=(n_prof, n))
    sups = set()
    atoms = np.zeros((n_atoms, n), np.int16)
    which = np.arange(n_atoms) % n_prof
    a = 0
    while a < n_atoms:
        s = tuple(sorted(rng.choice(n, size=support, replace=False).tolist()))
        if s in sups:
            continue
        sups.add(s)
        idx = list(s)
        atoms[a, idx] = rng.integers(1, mag + 1, size=support) * prof[which[a], idx]
        a += 1
    groups = [np.flatnonzero(which == p) for p in range(n_prof)]
    pr = rng.integers(0, n_prof, size=n_sums)
    S = np.empty((n_sums, n), np.int8)
    for p in range(n_prof):
        rows = np.flatnonzero(pr == p)
        i = rng.choice(groups[p], size=rows.size)
        j = rng.choice(groups[p], size=rows.size)
        j = np.where(i == j, groups[p][(np.searchsorted(groups[p], j) + 1) % groups[p].size], j)
        S[rows] = (atoms[i] + atoms[j]).astype(np.int8)
    X = np.concatenate([atoms.astype(np.int8), S])
    X = X[rng.permutation(X.shape[0])]
    neg = rng.random(X.shape[0]) < 0.5
    X[neg] = -X[neg]
    return X, atoms


def test_filter_closed_form_wide_index_and_magnitudes(G, ctx):
    """More than 2^21 distinct keys (the sign-pattern index then takes 13
    coordinates) with entries up to +-120, so the byte-wise magnitude test
    sees the whole int8 range the box allows."""
    X, atoms = _profile_set()
    _say("filter closed form profiles", X.shape, int(np.abs(X).max()))
    assert int(np.abs(X).max()) > 100
    want = sorted({canonical(tuple(int(v) for v in a)) for a in atoms})
    got = G.filter_minimal(ctx, torch.tensor(X, device="cuda"))
    assert got.shape[0] == len(want)
    assert _rows(got) == want


def test_filter_empty(G, ctx):
    got = G.filter_minimal(ctx, torch.zeros((0, 5), dtype=torch.int8, device="cuda"))
    assert got.shape[0] == 0


def _aug_case(kind):
    if kind == "tiny-int":
        inst = W.tiny_instance(1000)
        B = lattice.kernel_basis(inst.A)
        keys, _ = S.extract(inst.A, B, inst.l, inst.u, W.gaussian_starts(1024, B.shape[1], 2.0, 1001), 200,
                            S.AdamParams())
        F = np.array(o_filter(keys), dtype=np.int64)
        f = Objective("quadratic", Q=inst.Q, c=inst.c)
        S0 = 16
    elif kind == "qp-real":
        inst = W.qp_instance(2000)
        B = lattice.kernel_basis(inst.A)
        rng = np.random.default_rng(3)
        Z = rng.integers(-1, 2, size=(400, B.shape[1])) * (rng.random((400, B.shape[1])) < 0.05)
        G_ = Z @ B.T
        G_ = G_[np.all(np.abs(G_) <= 20, axis=1) & np.any(G_ != 0, axis=1)]
        F = np.array(sorted({canonical(g) for g in G_}), dtype=np.int64)
        f = Objective("quadratic", Q=inst.Q, c=inst.c)
        S0 = 6
    else:
        inst = W.quartic_instance(3000)
        B = lattice.kernel_basis(inst.A)
        rng = np.random.default_rng(5)
        Z = rng.integers(-1, 2, size=(300, B.shape[1])) * (rng.random((300, B.shape[1])) < 0.01)
        G_ = Z @ B.T
        G_ = G_[np.all(np.abs(G_) <= 40, axis=1) & np.any(G_ != 0, axis=1)]
        F = np.array(sorted({canonical(g) for g in G_}), dtype=np.int64)
        f = Objective("separable_poly", coef=inst.coef)
        S0 = 4
    starts = W.feasible_walk_starts(inst.x0, F, inst.l, inst.u, S0, seed=11, walk_len=16)
    return inst, F, f, starts


@pytest.mark.parametrize("kind", ["tiny-int", "qp-real", "quartic"])
def test_augment_bit_exact(G, ctx, kind):
    _say("augment", kind)
    inst, F, f, starts = _aug_case(kind)
    Xo, fo, so, bo = o_augment(inst.A, inst.b, inst.l, inst.u, f, F, starts)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, np.zeros((inst.n, 1), np.int64))
    obj = G.objective(f.kind, Q=f.Q, c=f.c, coef=f.coef)
    x, fv, steps, best = G.augment(ctx, prob, obj, torch.tensor(F.astype(np.int8), device="cuda"),
                                   torch.tensor(starts, device="cuda"))
    assert np.array_equal(x.cpu().numpy(), Xo)
    assert np.array_equal(steps.cpu().numpy(), so)
    assert np.array_equal(fv.cpu().numpy(), fo)
    assert best == bo
    _say("augment steps", kind, so.tolist())


def test_augment_errors_and_caps(G, ctx):
    _say("augment errors")
    inst, F, f, starts = _aug_case("tiny-int")
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, np.zeros((inst.n, 1), np.int64))
    obj = G.objective("quadratic", Q=inst.Q, c=inst.c)
    Fd = torch.tensor(F.astype(np.int8), device="cuda")
    bad = starts.copy()
    bad[1, 0] += 1
    with pytest.raises(G.GraverError) as e:
        G.augment(ctx, prob, obj, Fd, torch.tensor(bad, device="cuda"))
    assert e.value.status == -2
    Qa = inst.Q.copy()
    Qa[0, 1] += 1.0
    with pytest.raises(G.GraverError) as e:
        G.augment(ctx, prob, G.objective("quadratic", Q=Qa, c=inst.c), Fd, torch.tensor(starts, device="cuda"))
    assert e.value.status == -1
    Xo, fo, so, bo = o_augment(inst.A, inst.b, inst.l, inst.u, f, F, starts, max_steps=2)
    x, fv, steps, best = G.augment(ctx, prob, obj, Fd, torch.tensor(starts, device="cuda"), max_steps=2)
    assert np.array_equal(x.cpu().numpy(), Xo) and np.array_equal(steps.cpu().numpy(), so)
    x, fv, steps, best = G.augment(ctx, prob, obj, Fd[:0], torch.tensor(starts, device="cuda"))
    assert np.array_equal(x.cpu().numpy(), starts) and int(steps.sum()) == 0

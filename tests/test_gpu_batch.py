"""Batched extraction: many instances of uneven size in shared grids (one
per tile shape and forward form), optionally captured as a HIP graph.  With
the fixed shape table each instance's keys and final state equal a single
graver_extract call's bit for bit; with autotuning the sets are valid and
match the binary64 sets up to rounding-edge cases."""
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


# (n, m, N, precision, polish, pool capacity): identity-block instances of
# the batching law's size range; the shapes cover the tile shapes
# (1, 8), (1, 12), (2, 8), (2, 12) and the small-basis kernel.
SPECS = [
    (150, 30, 3000, "fp32", 0, 1 << 20),    # d = 120
    (210, 40, 1500, "fp32", 0, 1 << 20),    # d = 170
    (260, 60, 2200, "bf16", 20, 1 << 20),   # d = 200
    (420, 60, 700, "fp32", 0, 1 << 20),     # d = 360
    (340, 90, 900, "bf16", 0, 1 << 20),     # d = 250
    (100, 20, 4000, "fp32", 0, 1 << 20),    # small kernel
]

_cache = {}


def _batch(G):
    if "b" not in _cache:
        items = []
        for k, (n, m, N, prec, pol, cap) in enumerate(SPECS):
            inst = W.identity_block_instance(7000 + k, n, m)
            B = lattice.kernel_basis(inst.A, lll=False)
            z0 = W.gaussian_starts(N, B.shape[1], 0.3, 100 + k)
            items.append((inst, B, z0, prec, pol, cap))
        _cache["b"] = items
    return _cache["b"]


def _params(G, item, T=60, cap=None, form=None):
    """Matrix-core forms by default (the shared grids and their tile shapes
    are what these tests cover); form=GRAVER_FORM_AUTO lets the binary32
    instances, whose bases are sparse, take the sparse form (run alone)."""
    inst, B, z0, prec, pol, pcap = item
    p = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
    return G.extract_params(z0.shape[0], T, precision=p, init_mode=1, polish_iters=pol,
                            pool_capacity=pcap if cap is None else cap,
                            form=G.GRAVER_FORM_DENSE if form is None else form)


def _state(item):
    z0 = item[2]
    dev = lambda x: torch.tensor(x, dtype=torch.float64, device="cuda")
    return {"z": dev(z0), "m": dev(np.zeros_like(z0)), "v": dev(np.zeros_like(z0))}


@pytest.mark.parametrize("graph", [False, True], ids=["streams", "graph"])
def test_batch_equals_single_calls(G, graph):
    items = _batch(G)
    ctx = G.Context(0)
    probs = [G.DeviceProblem.from_numpy(it[0].A, it[0].b, it[0].l, it[0].u, it[1]) for it in items]
    prms = [_params(G, it) for it in items]
    states = [_state(it) for it in items]
    keys, stats, bs = G.extract_batch(ctx, probs, prms, states, autotune=False, use_graph=graph)
    _say("batch", "graph" if graph else "streams", bs, [s["unique"] for s in stats])
    assert bs["launches"] >= 1 and (bs["graphs"] >= 1) == graph
    single = G.Context(0)
    for i, it in enumerate(items):
        st = _state(it)
        k1, s1 = G.extract(single, probs[i], _params(G, it), state=st)
        if not torch.equal(keys[i], k1):
            a = keys[i].cpu().numpy()
            b = k1.cpu().numpy()
            sa, sb = {r.tobytes() for r in a}, {r.tobytes() for r in b}
            rows = int((a != b).any(axis=1).sum()) if a.shape == b.shape else -1
            raise AssertionError(f"instance {i}: keys differ: counts {a.shape[0]} {b.shape[0]}, "
                                 f"sets equal {sa == sb}, |a-b| {len(sa - sb)}, |b-a| {len(sb - sa)}, "
                                 f"rows differing {rows}, stats batch {stats[i]} single {s1}")
        assert torch.equal(states[i]["z"], st["z"]) and torch.equal(states[i]["m"], st["m"])
        assert s1["inbox_events"] == stats[i]["inbox_events"]
        K = keys[i].cpu().numpy().astype(np.int64)
        assert K.shape[0] > 0 and np.all(K @ it[0].A.T == 0)
    ctx.close()
    single.close()


def test_batch_with_sparse_form_instances_equals_single_calls(G):
    """The binary32 instances take the sparse form (alone, outside the shared
    grids) next to the bf16 instances' shared grids: every instance's keys,
    final state and event count equal a single call's."""
    items = _batch(G)
    ctx = G.Context(0)
    auto = G.GRAVER_FORM_AUTO
    probs = [G.DeviceProblem.from_numpy(it[0].A, it[0].b, it[0].l, it[0].u, it[1]) for it in items]
    prms = [_params(G, it, form=auto) for it in items]
    states = [_state(it) for it in items]
    keys, stats, bs = G.extract_batch(ctx, probs, prms, states, use_graph=True)
    _say("batch sparse", bs, [s["row_entries"] for s in stats])
    assert sum(s["row_entries"] > 0 for s in stats) >= 2
    single = G.Context(0)
    for i, it in enumerate(items):
        st = _state(it)
        k1, s1 = G.extract(single, probs[i], _params(G, it, form=auto), state=st)
        assert torch.equal(keys[i], k1)
        assert torch.equal(states[i]["z"], st["z"]) and torch.equal(states[i]["m"], st["m"])
        assert s1["inbox_events"] == stats[i]["inbox_events"]
    ctx.close()
    single.close()


def test_batch_log_overflow_replays_alone(G):
    """An instance whose log overflows in the shared grid is rolled back and
    replayed alone; its set equals a single call with a large pool."""
    items = _batch(G)
    ctx = G.Context(0)
    probs = [G.DeviceProblem.from_numpy(it[0].A, it[0].b, it[0].l, it[0].u, it[1]) for it in items]
    ref_ctx = G.Context(0)
    k_ref, s_ref = G.extract(ref_ctx, probs[1], _params(G, items[1]), state=_state(items[1]))
    cap = k_ref.shape[0]
    assert s_ref["inbox_events"] > cap
    prms = [_params(G, it) for it in items]
    prms[1] = _params(G, items[1], cap=cap)
    keys, stats, bs = G.extract_batch(ctx, probs, prms, [_state(it) for it in items], use_graph=True)
    _say("batch overflow", bs, "unique", cap)
    assert bs["replays"] >= 1
    assert torch.equal(keys[1], k_ref)
    ctx.close()
    ref_ctx.close()


def test_batch_autotuned_sets_valid(G):
    items = _batch(G)
    ctx = G.Context(0)
    probs = [G.DeviceProblem.from_numpy(it[0].A, it[0].b, it[0].l, it[0].u, it[1]) for it in items]
    prms = [_params(G, it) for it in items]
    keys, stats, bs = G.extract_batch(ctx, probs, prms, [_state(it) for it in items], autotune=True,
                                      use_graph=True)
    _say("batch autotuned", bs)
    for i, it in enumerate(items):
        k64, _ = G.extract(ctx, probs[i], G.extract_params(it[2].shape[0], 60, precision=G.GRAVER_FP64,
                                                           init_mode=1, pool_capacity=1 << 20),
                           state={"z": torch.tensor(it[2], dtype=torch.float64, device="cuda")})
        a = {tuple(r) for r in keys[i].cpu().numpy().tolist()}
        b = {tuple(r) for r in k64.cpu().numpy().tolist()}
        jac = len(a & b) / max(1, len(a | b))
        _say("batch autotuned", i, len(a), len(b), "jaccard", jac)
        assert jac >= 0.9
        K = keys[i].cpu().numpy().astype(np.int64)
        assert np.all(K @ it[0].A.T == 0) and np.all(np.abs(K) <= (it[0].u - it[0].l)[None, :])
    ctx.close()

"""The largest single-GPU configuration at its full size, checked on sampled
outputs: the quartic workload (m = 50, n = 400, d = 350), 262144 box starts
x 2000 binary32 iterations (about 9.5e7 distinct candidates), then the
minimality filter over all of them.  Sampled keys are in the box and satisfy
A g = 0 exactly; sampled survivors of the filter have no conformally smaller
element in X u -X and sampled removed keys have one (exact int8 compares over
the whole set on the device).  This is also the size at which a row mover
with a thread per word exceeds the 2^32 - 1 work-items of one dispatch."""
import numpy as np
import pytest

from paper_2412_13576_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2412_13576_amd import graver
    return graver


def _has_witness(keys, g):
    """Some h in X u -X, h != +-g, with h_i g_i >= 0 and |h_i| <= |g_i|."""
    lo = torch.minimum(g, torch.zeros_like(g))
    hi = torch.maximum(g, torch.zeros_like(g))
    for c0 in range(0, keys.shape[0], 1 << 22):
        X = keys[c0:c0 + (1 << 22)]
        pos = ((X >= lo) & (X <= hi)).all(dim=1)
        neg = ((X >= -hi) & (X <= -lo)).all(dim=1)
        same = (X == g).all(dim=1) | (X == -g).all(dim=1)
        if ((pos | neg) & ~same).any():
            return True
    return False


def test_quartic_full_size_extraction_and_filter(G):
    inst = W.quartic_instance()
    B, P = G.kernel_basis(inst.A)
    N, T = 262144, 2000
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, B, P)
    _say("full scale extraction", N, T)
    prm = G.extract_params(N, T, precision=G.GRAVER_FP32, init_mode=0, seed=3, pool_capacity=500 * N,
                           any_order=True)
    keys, st = G.extract(ctx, prob, prm)
    K = int(keys.shape[0])
    _say("full scale", {k: st[k] for k in ("emit_events", "inbox_events", "unique", "out_of_range")})
    assert K == st["unique"] == st["verified"] > 50_000_000 and st["out_of_range"] == 0
    rng = np.random.default_rng(0)
    sample = keys[torch.as_tensor(rng.choice(K, size=4096, replace=False), device="cuda")].cpu().numpy()
    S64 = sample.astype(np.int64)
    assert not np.any(inst.A @ S64.T)
    assert np.all(np.abs(S64) <= (inst.u - inst.l)[None, :]) and np.all(np.any(S64 != 0, axis=1))
    ctx.trim()
    F = G.filter_minimal(ctx, keys)
    ctx.trim()
    R = int(F.shape[0])
    _say("full scale filter", K, "->", R)
    assert 0 < R < K
    # canonical (first nonzero positive) and strictly increasing
    Fs = F[torch.as_tensor(np.sort(rng.choice(R, size=2048, replace=False)), device="cuda")].cpu().numpy()
    first = Fs[np.arange(Fs.shape[0]), np.argmax(Fs != 0, axis=1)]
    assert np.all(first > 0)
    for g in F[torch.as_tensor(rng.choice(R, size=24, replace=False), device="cuda")]:
        assert not _has_witness(keys, g)
    # removed keys: canonical forms of sampled keys that are not in F
    Fv = np.ascontiguousarray(F.cpu().numpy()).view(np.dtype((np.void, F.shape[1]))).ravel()
    idx = rng.choice(K, size=20000, replace=False)
    cand = keys[torch.as_tensor(idx, device="cuda")].cpu().numpy()
    fc = cand[np.arange(cand.shape[0]), np.argmax(cand != 0, axis=1)]
    cand = np.where(fc[:, None] < 0, -cand, cand).astype(np.int8)
    cv = np.ascontiguousarray(cand).view(np.dtype((np.void, cand.shape[1]))).ravel()
    removed = cand[~np.isin(cv, Fv)][:24]
    assert removed.shape[0] > 0
    for g in removed:
        assert _has_witness(keys, torch.as_tensor(g, device="cuda"))
    ctx.close()

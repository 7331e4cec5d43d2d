"""The request server: continuous batching of MAPE requests (Section 3.3).
A request's answer is the same alone and in a mix of other requests (bit
for bit, fixed tile shapes), equals graver_solve with the same parameters,
and every request completes under a tiny device-memory budget."""
import numpy as np
import pytest

from oracle import augment as AG
from paper_2412_13576_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_2412_13576_amd import graver
    return graver


# (seed, n, m, precision, objective): identity-block instances, quadratic or
# quartic (separable degree 4 with coefficients drawn like the quartic law)
MIX = [(11, 60, 12, "fp32", "quad"), (12, 150, 30, "bf16", "quartic"), (13, 90, 18, "fp32", "quad"),
       (14, 250, 50, "fp32", "quartic"), (15, 180, 36, "bf16", "quad"), (16, 40, 8, "fp32", "quad"),
       (17, 320, 64, "fp32", "quad")]


def _request(G, seed, n, m, prec, kind, T=200):
    inst = W.identity_block_instance(seed, n, m)
    N = 16 * n
    p = G.GRAVER_FP32 if prec == "fp32" else G.GRAVER_BF16
    ex = G.extract_params(N, T, precision=p, init_mode=0, seed=seed, pool_capacity=32 * N,
                          polish_iters=T // 10 if prec == "bf16" else 0)
    ini = G.init_params(8, 200, seed=seed + 1, lr=0.05)
    obj = {}
    if kind == "quad":
        obj = dict(Q=inst.Q, c=inst.c)
    else:
        rng = np.random.default_rng(seed)
        coef = np.zeros((n, 5))
        coef[:, 4] = rng.uniform(0.1, 1.0, n)
        coef[:, 3] = rng.standard_normal(n)
        coef[:, 2] = rng.standard_normal(n)
        obj = dict(coef=coef)
    return inst, ex, ini, obj


def _submit(G, srv, item):
    inst, ex, ini, obj = item
    return srv.submit(inst.A, inst.b, inst.l, inst.u, ex, ini, lll=False, x_starts=inst.x0[None, :], **obj)


def test_server_alone_equals_mix_equals_solve(G):
    items = [_request(G, *spec) for spec in MIX]
    target = 3
    srv = G.Server(max_batch=8, gpu_workers=2, host_threads=4, batch_window_us=200000)
    alone, xa = srv.wait(_submit(G, srv, items[target]))
    _say("server alone", alone)
    assert alone["status"] == 0 and alone["batch_size"] == 1
    tickets = [_submit(G, srv, it) for it in items]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    mixed, xm = res[target]
    _say("server mix", [(r["batch_size"], r["status"], round(r["t_done"] - r["t_submit"], 3)) for r, _ in res])
    assert all(r["status"] == 0 for r, _ in res)
    assert max(r["batch_size"] for r, _ in res) > 1
    assert mixed["f_best"] == alone["f_best"] and np.array_equal(xm, xa)
    assert mixed["unique"] == alone["unique"] and mixed["filtered"] == alone["filtered"]
    # the same request through graver_solve
    inst, ex, ini, obj = items[target]
    ctx = G.Context(0)
    prob = G.DeviceProblem.from_numpy(inst.A, inst.b, inst.l, inst.u, None)
    o = G.objective("quadratic", **obj) if "Q" in obj else G.objective("poly", coef=obj["coef"])
    sp = G.solve_params(ex, ini, reuse=False, lll=False, x_starts=torch.tensor(inst.x0[None, :], device="cuda"))
    x, fb, st = G.solve(ctx, prob, o, sp)
    ctx.close()
    _say("server vs solve", fb, alone["f_best"], st["unique"], alone["unique"])
    assert fb == alone["f_best"] and np.array_equal(x.cpu().numpy(), xa)
    # the answer is feasible and its objective is the oracle's objective of it
    f = AG.Objective("quadratic", Q=inst.Q, c=inst.c) if "Q" in obj else AG.Objective("separable_poly",
                                                                                       coef=obj["coef"])
    assert np.all(inst.A @ xa == inst.b) and np.all((xa >= inst.l) & (xa <= inst.u))
    assert np.float64(alone["f_best"]).view(np.uint64) == np.float64(AG.objective(f, xa)).view(np.uint64)


def test_server_tiny_budget_and_errors(G):
    """With a budget below any request's footprint every request is admitted
    alone (and still completes); a request without any feasible start fails
    alone."""
    items = [_request(G, *spec, T=60) for spec in MIX[:4]]
    srv = G.Server(hbm_budget=1, max_batch=8, gpu_workers=2, host_threads=2)
    tickets = [_submit(G, srv, it) for it in items]
    inst, ex, ini, obj = items[0]
    bad = srv.submit(inst.A, inst.b + 1000, inst.l, inst.u, ex, G.init_params(2, 5), Q=inst.Q, c=inst.c, lll=False)
    res = [srv.wait(t) for t in tickets]
    rb, xb = srv.wait(bad)
    srv.close()
    _say("server tiny budget", [(r["batch_size"], r["status"]) for r, _ in res], "bad", rb["status"])
    assert all(r["status"] == 0 and r["batch_size"] == 1 for r, _ in res)
    assert rb["status"] == G.GRAVER_E_INFEASIBLE_START and xb is None


def test_server_poll_and_cancel(G):
    """Poll before and after completion; cancel a request still queued for its
    basis (one basis thread busy with an LLL basis) and one already running
    on the GPU; the server keeps serving afterwards."""
    import time
    srv = G.Server(max_batch=4, gpu_workers=1, host_threads=1)
    slow = W.identity_block_instance(21, 300, 60)
    ex = G.extract_params(16 * 300, 100, precision=G.GRAVER_FP32, init_mode=0, seed=21, pool_capacity=1 << 16)
    ini = G.init_params(4, 50, seed=22, lr=0.05)
    ta = srv.submit(slow.A, slow.b, slow.l, slow.u, ex, ini, Q=slow.Q, c=slow.c, lll=True,
                    x_starts=slow.x0[None, :])
    item_b = _request(G, 23, 40, 8, "fp32", "quad", T=50)
    tb = _submit(G, srv, item_b)
    assert srv.cancel(tb)  # the only basis thread is still reducing the first basis
    done, ra, _ = srv.poll(ta)
    assert not done
    rb, xb = srv.wait(tb)
    _say("cancelled queued", rb["status"], rb["batch_size"])
    assert rb["status"] == G.GRAVER_E_CANCELLED and xb is None and rb["batch_size"] == 0
    t0 = time.time()
    while True:
        done, ra, xa = srv.poll(ta)
        if done:
            break
        assert time.time() - t0 < 120
        time.sleep(0.05)
    assert ra["status"] == 0 and xa is not None
    srv.n[ta] = slow.n
    with pytest.raises(G.GraverError):  # released by the poll that returned it
        srv.cancel(ta)
    # a long extraction, cancelled while it runs on the GPU
    exl = G.extract_params(16 * 300, 100000, precision=G.GRAVER_FP32, init_mode=0, seed=24, pool_capacity=1 << 21)
    tl = srv.submit(slow.A, slow.b, slow.l, slow.u, exl, ini, Q=slow.Q, c=slow.c, lll=True,
                    x_starts=slow.x0[None, :])
    time.sleep(0.5)
    assert srv.cancel(tl)
    rl, xl = srv.wait(tl)
    _say("cancelled running", rl["status"], rl["batch_size"], round(rl["t_done"] - rl["t_submit"], 2))
    assert rl["status"] == G.GRAVER_E_CANCELLED and xl is None
    # the server still serves
    rc, xc = srv.wait(_submit(G, srv, _request(G, 25, 60, 12, "fp32", "quad", T=60)))
    srv.close()
    assert rc["status"] == 0 and xc is not None

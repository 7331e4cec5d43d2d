"""Pins for the oracle of eq. init_sol (initial feasible solutions)."""
import numpy as np
import pytest

from oracle import init_sol as I
from oracle.surrogate import AdamParams
from paper_2412_13576_amd import workloads as W

P = AdamParams()


def test_gradient_matches_finite_differences():
    inst = W.tiny_instance(1000)
    rng = np.random.default_rng(0)
    done = 0
    for _ in range(40):
        x = rng.uniform(-4, 4, size=(1, 8))
        frac = x - np.floor(x)
        if np.minimum(frac, 1 - frac).min() < 1e-3:
            continue
        g = I.grad_init(inst.A, inst.b, x, 0.1)[0]
        h = 1e-6
        for j in range(8):
            e = np.zeros_like(x)
            e[0, j] = h
            fd = (I.objective_init(inst.A, inst.b, x + e, 0.1) - I.objective_init(inst.A, inst.b, x - e, 0.1))[0] / (2 * h)
            assert abs(fd - g[j]) <= 1e-5 * max(1.0, abs(fd))
        done += 1
    assert done >= 10


def test_identity_system_converges_to_b():
    # A = I: the unique feasible integer point is b; from any start in the
    # box projected Adam approaches it and rounding recovers it exactly.
    n = 6
    A = np.eye(n, dtype=np.int64)
    b = np.array([2, -1, 0, 3, -3, 1])
    l, u = np.full(n, -4), np.full(n, 4)
    x0 = I.box_uniform_starts(l, u, 32, seed=3)
    x, r, feas = I.init_solutions(A, b, l, u, x0, 3000, AdamParams(lr=0.01), lam3=0.1)
    assert np.all(feas) and np.all(r == b[None, :])
    assert np.all(x >= l) and np.all(x <= u)


def test_projection_and_feasibility_flags_on_tiny_instance():
    inst = W.tiny_instance(1001)
    x0 = I.box_uniform_starts(inst.l, inst.u, 200, seed=5)
    x, r, feas = I.init_solutions(inst.A, inst.b, inst.l, inst.u, x0, 1500, AdamParams(lr=0.01))
    assert np.all(x >= inst.l) and np.all(x <= inst.u)
    assert np.any(feas)
    for k in np.nonzero(feas)[0]:
        assert np.all(inst.A @ r[k] == inst.b)


def test_matches_torch_projected_adam():
    torch = pytest.importorskip("torch")
    inst = W.tiny_instance(1002)
    x0 = I.box_uniform_starts(inst.l, inst.u, 64, seed=9)
    xo, _, _ = I.init_solutions(inst.A, inst.b, inst.l, inst.u, x0, 40, P)
    A = torch.tensor(inst.A, dtype=torch.float64)
    b = torch.tensor(inst.b, dtype=torch.float64)
    x = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=P.lr, betas=(P.beta1, P.beta2), eps=P.eps)
    lo = torch.tensor(inst.l, dtype=torch.float64)
    hi = torch.tensor(inst.u, dtype=torch.float64)
    for _ in range(40):
        opt.zero_grad()
        r = x @ A.T - b
        loss = ((r * r).sum(1) + 0.1 * ((x - torch.floor(x)) * (torch.ceil(x) - x)).sum(1)).sum()
        loss.backward()
        opt.step()
        with torch.no_grad():
            x.copy_(torch.minimum(torch.maximum(x, lo), hi))
    err = np.abs(x.detach().numpy() - xo).max(axis=1)
    assert np.mean(err < 1e-9) >= 0.95

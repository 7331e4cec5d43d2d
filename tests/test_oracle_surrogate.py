"""Pins for the surrogate Phi, its gradient, Adam and Parallel Extraction
(Section 3.2, eq. loss, Algorithm 2) and the Philox start generator."""
import numpy as np
import pytest

from oracle import lattice, philox
from oracle import surrogate as S
from oracle.conformal import graver_basis_in_box, in_kernel, kernel_vectors_in_box
from paper_2412_13576_amd import workloads as W
from tests.golden_io import philox_kat

P = S.AdamParams()


def _inst_basis():
    inst = W.tiny_instance(1000)
    return inst, lattice.kernel_basis(inst.A)


def test_gradient_matches_finite_differences_away_from_kinks():
    inst, B = _inst_basis()
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(60):
        z = rng.normal(0, 0.8, size=(1, B.shape[1]))
        y = z @ B.T
        frac = z - np.floor(z)
        if np.abs(y).min() < 1e-3 or np.minimum(frac, 1 - frac).min() < 1e-3:
            continue
        az = np.abs(z)
        if np.sort(az.ravel())[-1] - np.sort(az.ravel())[-2] < 1e-3 or abs(az.max() - 1) < 1e-3:
            continue
        g = S.grad_phi(B.astype(float), z, P.lambda1, P.lambda2)[0]
        h = 1e-6
        for j in range(B.shape[1]):
            e = np.zeros_like(z)
            e[0, j] = h
            fd = (S.phi(B, z + e, P.lambda1, P.lambda2) - S.phi(B, z - e, P.lambda1, P.lambda2))[0] / (2 * h)
            assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd))
        checked += 1
    assert checked >= 10


def test_phi_is_even_and_trajectories_negate_exactly():
    inst, B = _inst_basis()
    z0 = W.gaussian_starts(32, B.shape[1], 2.0, 1001)
    assert np.array_equal(S.phi(B, z0, 0.85, 1.0), S.phi(B, -z0, 0.85, 1.0))
    za, ma, va, _ = S.descend(B, z0, 50, P)
    zb, mb, vb, _ = S.descend(B, -z0, 50, P)
    assert np.array_equal(za, -zb) and np.array_equal(ma, -mb) and np.array_equal(va, vb)


def test_phi_at_integer_points_is_l1_norm():
    inst, B = _inst_basis()
    rng = np.random.default_rng(4)
    z = rng.integers(-3, 4, size=(50, B.shape[1])).astype(float)
    z = z[np.abs(z).max(axis=1) >= 1]
    assert np.array_equal(S.phi(B, z, 0.85, 1.0), np.abs(z @ B.T).sum(axis=1))


def test_adam_first_step_is_signed_learning_rate():
    inst, B = _inst_basis()
    z0 = W.gaussian_starts(16, B.shape[1], 2.0, 7)
    g = S.grad_phi(B.astype(float), z0, P.lambda1, P.lambda2)
    z1, _, _, _ = S.descend(B, z0, 1, P)
    # m_hat = g and v_hat = g^2 after one step, so dz = -lr g / (|g| + eps)
    expect = -P.lr * g / (np.abs(g) + P.eps)
    assert np.allclose(z1 - z0, expect, rtol=1e-12, atol=1e-15)


def test_barrier_gradient_split_over_ties():
    B = np.eye(3, dtype=np.int64)
    z = np.array([[0.5, -0.5, 0.25]])
    g = S.grad_phi(B.astype(float), z, 0.0, 1.0)[0]
    # d/dz_k of (1/mu - 1) with mu = 0.5 shared by two coordinates
    expect_bar = np.array([-1.0 / (0.25 * 2), 1.0 / (0.25 * 2), 0.0])
    assert np.allclose(g - np.sign(z[0]), expect_bar)


def test_extract_outputs_satisfy_conditions_and_are_graver_heavy():
    inst, B = _inst_basis()
    z0 = W.gaussian_starts(256, B.shape[1], 2.0, 1001)
    keys, _ = S.extract(inst.A, B, inst.l, inst.u, z0, 300, P)
    assert len(keys) > 0
    R = inst.u - inst.l
    for g in keys:
        assert any(g) and in_kernel(inst.A, g)
        assert all(abs(x) <= r for x, r in zip(g, R))
    assert keys == sorted(set(keys))
    # every collected vector is a kernel vector of the box; report recall
    Gb = set(graver_basis_in_box(inst.A, 6))
    assert len(Gb & set(keys)) > 0


def test_extract_skip_unchanged_is_equivalent():
    inst, B = _inst_basis()
    z0 = W.gaussian_starts(64, B.shape[1], 2.0, 99)
    keys, _ = S.extract(inst.A, B, inst.l, inst.u, z0, 120, P)
    # plain Algorithm 2: round and collect after every step, no skipping
    Bf = B.astype(float)
    z, m, v = z0.copy(), np.zeros_like(z0), np.zeros_like(z0)
    found = set()
    for t in range(1, 121):
        z, m, v = S.adam_step(z, m, v, S.grad_phi(Bf, z, P.lambda1, P.lambda2), t, P)
        gs = np.rint(z).astype(np.int64) @ B.T
        for g in gs[S.in_box(gs, inst.l, inst.u)]:
            found.add(tuple(int(x) for x in g))
    assert keys == sorted(found)


def test_extract_resume_equals_single_run():
    inst, B = _inst_basis()
    z0 = W.gaussian_starts(32, B.shape[1], 2.0, 5)
    k_all, (z_all, _, _) = S.extract(inst.A, B, inst.l, inst.u, z0, 80, P)
    k1, (z1, m1, v1) = S.extract(inst.A, B, inst.l, inst.u, z0, 30, P)
    k2, (z2, _, _) = S.extract(inst.A, B, inst.l, inst.u, z1, 50, P, m0=m1, v0=v1, t0=30)
    assert np.array_equal(z2, z_all)
    assert set(k_all) == set(k1) | set(k2)


@pytest.mark.parametrize("ctr,key,out", philox_kat())
def test_philox_known_answers(ctr, key, out):
    got = philox.philox4x32_10(tuple([c] for c in ctr), tuple(key))
    assert [int(w[0]) for w in got] == out


def test_box_starts_distribution_and_projection():
    inst, B = _inst_basis()
    Pm = lattice.coordinate_projector(B)
    g, z = philox.box_starts(Pm, inst.l, inst.u, 4000, seed=12)
    lo, hi = inst.l - inst.u, inst.u - inst.l
    assert np.all(g >= lo) and np.all(g < hi)
    assert abs(g.mean()) < 0.3 and abs(g.var() - (hi[0] - lo[0]) ** 2 / 12) < 2.0
    assert np.allclose(z, g @ Pm.T, rtol=1e-12, atol=1e-12)
    g2, _ = philox.box_starts(Pm, inst.l, inst.u, 10, seed=12, first_start=5)
    assert np.array_equal(g2[:5], g[5:10])


def test_descent_matches_torch_autograd_and_adam():
    """The same descent through an independent implementation: torch
    autograd of eq. loss (abs'(0) = 0, zero derivative of floor/ceil, amax
    gradient split over ties) and torch.optim.Adam (Kingma and Ba), in
    float64 on the CPU."""
    torch = pytest.importorskip("torch")
    inst, B = _inst_basis()
    z0 = W.gaussian_starts(64, B.shape[1], 2.0, 31)
    zo, _, _, _ = S.descend(B, z0, 40, P)
    Bt = torch.tensor(B, dtype=torch.float64)
    z = torch.tensor(z0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([z], lr=P.lr, betas=(P.beta1, P.beta2), eps=P.eps)
    for _ in range(40):
        opt.zero_grad()
        y = z @ Bt.T
        mu = torch.amax(z.abs(), dim=1)
        loss = (y.abs().sum(1) + P.lambda1 * ((z - torch.floor(z)) * (torch.ceil(z) - z)).sum(1)
                + P.lambda2 * torch.clamp(1.0 / mu - 1.0, min=0.0)).sum()
        loss.backward()
        opt.step()
    zt = z.detach().numpy()
    err = np.abs(zt - zo).max(axis=1) / np.maximum(np.abs(zo).max(axis=1), 1.0)
    # a start whose trajectory crossed a kink may split; nearly all must agree
    assert np.mean(err < 1e-9) >= 0.95

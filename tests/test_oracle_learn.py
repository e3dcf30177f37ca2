"""Pins of the learned-weight oracle (oracle/learn.py) against closed forms,
library routines and finite differences."""
import numpy as np
import pytest

import oracle
from oracle import learn as ol

torch = pytest.importorskip("torch")


def lattice(rho, n, sub=None):
    """One point at the centre of every cell of an n^3 grid over [-rho, rho]^3
    (or of the cells with all indices < sub)."""
    h = 2.0 * rho / n
    k = np.arange(n if sub is None else sub)
    a = -rho + (k + 0.5) * h
    x, y, z = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def test_features_uniform_lattice_is_the_cube_density():
    # one point per cell of the finest grid: every histogram sees density 1 / (2 rho)^3
    rho = 2.5
    pts = lattice(rho, 64)
    f = ol.features(pts, rho)
    assert np.allclose(f[:, :3], -3.0 * np.log(2.0 * rho), atol=1e-12, rtol=0)
    assert np.allclose(f[:, 3], np.sum(pts ** 2, axis=1) / rho ** 2, rtol=1e-15)


def test_features_octant_lattice():
    # the octant of cells with indices < 32 only: density 1 / rho^3 inside it
    rho = 1.5
    pts = lattice(rho, 64, sub=32)
    f = ol.features(pts, rho)
    assert np.allclose(f[:, :3], -3.0 * np.log(rho), atol=1e-12, rtol=0)


def test_features_two_densities():
    # doubling the points of one half doubles the density there
    rho = 1.0
    pts = lattice(rho, 64)
    dup = pts[pts[:, 0] < 0]
    allp = np.concatenate([pts, dup])
    f = ol.features(allp, rho)
    M = allp.shape[0]
    lo = np.log(2.0 / (M * (2 * rho / 64) ** 3))
    hi = np.log(1.0 / (M * (2 * rho / 64) ** 3))
    neg = allp[:, 0] < 0
    assert np.allclose(f[neg, :3], lo, atol=1e-12) and np.allclose(f[~neg, :3], hi, atol=1e-12)


def test_weights_reduce_to_the_midpoint_rule_on_the_grid():
    # c = 0 on a uniform lattice: w_i = h^3 e^{-|x_i|^2}, the mid-point rule (Section 8)
    rho = 3.0
    pts = lattice(rho, 64)
    f = ol.features(pts, rho)
    w = ol.weights(np.zeros(len(pts)), f, rho)
    h = 2 * rho / 64
    assert np.allclose(w, h ** 3 * np.exp(-np.sum(pts ** 2, axis=1)), rtol=1e-12)


def random_params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, ol.num_params())


def test_mlp_matches_torch_layers():
    rng = np.random.default_rng(1)
    p = random_params(2)
    x = rng.standard_normal((50, 4))
    W1, b1, W2, b2, W3, b3 = ol.unpack(p)
    net = torch.nn.Sequential(torch.nn.Linear(4, 64), torch.nn.Tanh(), torch.nn.Linear(64, 64), torch.nn.Tanh(),
                              torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(W1)); net[0].bias.copy_(torch.from_numpy(b1))
        net[2].weight.copy_(torch.from_numpy(W2)); net[2].bias.copy_(torch.from_numpy(b2))
        net[4].weight.copy_(torch.from_numpy(W3[None, :])); net[4].bias.fill_(float(b3))
        ref = net(torch.from_numpy(x)).numpy()[:, 0]
    assert np.allclose(ol.mlp(p, x), ref, rtol=1e-13, atol=1e-13)


def test_mlp_grad_central_differences():
    rng = np.random.default_rng(3)
    p = random_params(4)
    x = rng.standard_normal((20, 4))
    dc = rng.standard_normal(20)
    g = ol.mlp_grad(p, x, dc)
    idx = rng.choice(len(p), 60, replace=False)
    idx = np.concatenate([idx, [0, 3, 256, 300, 320 + 64 * 64 - 1, len(p) - 65, len(p) - 1]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (dc @ ol.mlp(p + e, x) - dc @ ol.mlp(p - e, x)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * (1 + abs(g[k])), (k, fd, g[k])


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(30)
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(30), np.zeros(30)
    for step in range(1, 5):
        g = rng.standard_normal(30)
        t.grad = torch.tensor(g)
        opt.step()
        p, m, v = ol.adam(p, g, m, v, 1e-2, step)
        assert np.allclose(p, t.detach().numpy(), rtol=1e-14, atol=1e-14)


def test_loss_gradient_central_differences():
    B, M = 3, 40
    rng = np.random.default_rng(6)
    pts = rng.standard_normal((M, 3)) * 0.7
    fhats = [rng.standard_normal(oracle.num_coeffs(B)) + 1j * rng.standard_normal(oracle.num_coeffs(B))
             for _ in range(2)]

    def fwd(fh):
        return oracle.direct_forward(B, pts, fh)

    def adj(y):
        return oracle.direct_adjoint(B, pts, y)

    rho = 1.01 * np.sqrt(np.max(np.sum(pts ** 2, axis=1)))
    feat = ol.features(pts, rho)
    c = rng.standard_normal(M) * 0.3
    L, dc = ol.loss_and_dc(fwd, adj, ol.weights(c, feat, rho), fhats)
    h = 1e-6
    for i in range(0, M, 3):
        e = np.zeros(M)
        e[i] = h
        lp = ol.loss_and_dc(fwd, adj, ol.weights(c + e, feat, rho), fhats)[0]
        lm = ol.loss_and_dc(fwd, adj, ol.weights(c - e, feat, rho), fhats)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dc[i]) <= 1e-6 * (abs(L) + abs(dc[i])), (i, fd, dc[i])


def test_loss_is_zero_for_an_exact_quadrature():
    # B = 1: a single constant basis function; weights summing it exactly give L = 0
    B, M = 1, 30
    rng = np.random.default_rng(7)
    pts = rng.standard_normal((M, 3))
    fh = [np.array([1.0 + 0.5j])]
    y0 = oracle.direct_forward(B, pts, np.array([1.0 + 0j]))
    w = np.full(M, 1.0 / np.sum(np.abs(y0) ** 2))
    L, _ = ol.loss_and_dc(lambda f: oracle.direct_forward(B, pts, f), lambda y: oracle.direct_adjoint(B, pts, y),
                          w, fh)
    assert L < 1e-28

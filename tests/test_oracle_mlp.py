"""Pins of the surrogate's CPU reference (oracle/mlp.py) against independent facts.

* Features: invariant under rigid motions of (particle, triangle), vertex
  relabelling and orientation; flags equal brute-force counts; the rotation
  maps the integral oracle's h-frame result onto its result for the
  canonical triangle (pins the rotation's sign and the orientation rule).
* bfloat16 rounding equals torch's round-to-nearest-even conversion.
* Network: forward equals torch's functional ops; the analytic gradient
  equals central finite differences of the loss and torch autograd.
* Adam equals torch.optim.Adam.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp


def random_geometry(n, seed):
    rng = np.random.default_rng(seed)
    px = rng.uniform(-1, 1, n)
    py = rng.uniform(-1, 1, n)
    tri = np.empty((6, n))
    for k in range(3):
        tri[2 * k] = px + rng.uniform(-1.8, 1.8, n) * 0.1
        tri[2 * k + 1] = py + rng.uniform(-1.8, 1.8, n) * 0.1
    return px, py, tri, 0.1


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(0).standard_normal(20000) * 10.0 ** np.random.default_rng(1).uniform(-5, 5, 20000)
    x = np.concatenate([x, [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -2.5]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_features_invariances():
    px, py, tri, h = random_geometry(400, 1)
    f0, _ = mlp.features(px, py, tri, h)
    rng = np.random.default_rng(2)
    th = rng.uniform(0, 2 * np.pi)
    c, s = np.cos(th), np.sin(th)
    shift = rng.uniform(-5, 5, 2)

    def move(x, y):
        return c * x - s * y + shift[0], s * x + c * y + shift[1]

    mpx, mpy = move(px, py)
    mtri = tri.copy()
    for k in range(3):
        mtri[2 * k], mtri[2 * k + 1] = move(tri[2 * k], tri[2 * k + 1])
    f1, _ = mlp.features(mpx, mpy, mtri, h)
    np.testing.assert_allclose(f1, f0, atol=1e-10)
    # relabelling and orientation
    for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1], [2, 1, 0]):
        ptri = np.concatenate([tri[2 * k:2 * k + 2] for k in perm])
        f2, _ = mlp.features(px, py, ptri, h)
        np.testing.assert_allclose(f2, f0, atol=1e-12)
    # mirror: a reflected configuration has the y features negated after canonicalisation
    rtri = tri.copy()
    rtri[1::2] = 2 * py - tri[1::2]
    f3, _ = mlp.features(px, py, rtri, h)
    np.testing.assert_allclose(f3[:, 0], f0[:, 0], atol=1e-12)


def test_features_flags_brute_force():
    px, py, tri, h = random_geometry(300, 3)
    f, _ = mlp.features(px, py, tri, h)
    t = np.linspace(0.0, 1.0, 20001)
    for q in range(300):
        v = np.array([[(tri[2 * k, q] - px[q]) / h, (tri[2 * k + 1, q] - py[q]) / h] for k in range(3)])
        inside = np.sum(np.hypot(v[:, 0], v[:, 1]) <= 1.0)
        cross = 0
        for k in range(3):
            pts = v[k][None, :] + t[:, None] * (v[(k + 1) % 3] - v[k])[None, :]
            r = np.hypot(pts[:, 0], pts[:, 1])
            cross += int(r.min() < 1.0 < r.max())
        assert f[q, 6] * 3 == inside
        assert f[q, 7] * 3 == cross, q


def test_features_rotation_convention_against_integrals():
    """rotate_in(result of the h-frame) == result for the canonical triangle."""
    px, py, tri, h = random_geometry(60, 4)
    f, rot = mlp.features(px, py, tri, h)
    for q in range(60):
        res = np.array(oracle.pair(0, h, px[q], py[q], tri[:, q], np.ones(1)))
        res[1:] *= h
        can = oracle.pair(0, 1.0, 0.0, 0.0, f[q, :6].copy(), np.ones(1))
        np.testing.assert_allclose(mlp.rotate_in(res[None, :], rot[q:q + 1])[0], can, atol=1e-11)
        np.testing.assert_allclose(mlp.rotate_back(np.array([list(can) + [0.0]]), rot[q:q + 1])[0], res,
                                   atol=1e-11)


def test_features_particle_at_vertex_uses_identity_rotation():
    tri = np.array([[0.0], [0.0], [0.05], [0.01], [0.02], [0.06]])
    f, rot = mlp.features(np.zeros(1), np.zeros(1), tri, 0.1)
    assert rot[0].tolist() == [1.0, 0.0]
    assert f[0, 0] == 0.0 and f[0, 1] == 0.0


def torch_forward(params, x):
    t = torch.tensor(params, dtype=torch.float64)
    a = torch.tensor(x, dtype=torch.float64)
    o = 0
    for li, (i, n) in enumerate(mlp.LAYERS):
        W = t[o:o + i * n].reshape(i, n)
        o += i * n
        b = t[o:o + n]
        o += n
        a = a @ W + b
        if li < len(mlp.LAYERS) - 1:
            u = torch.clamp(a, -4.0, 4.0)
            a = a * (0.5 + u * (0.25 - u.abs() / 32.0))
    return a


def test_activation_is_c1_and_its_derivative_matches():
    z = np.linspace(-6, 6, 24001)
    a = mlp.act(z)
    # limits: 0 far left, identity far right, continuous derivative across the joins at |z| = 4 and 0
    assert np.all(a[z <= -4] == 0.0) and np.allclose(a[z >= 4], z[z >= 4])
    fd = np.gradient(a, z)
    np.testing.assert_allclose(mlp.act_grad(z)[1:-1], fd[1:-1], atol=2e-4)
    for c in (-4.0, 0.0, 4.0):
        e = 1e-9
        assert abs(mlp.act_grad(c - e) - mlp.act_grad(c + e)) < 1e-8


def test_param_count():
    assert mlp.N_PARAMS == 8 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 4 + 4 == 34692


def test_forward_matches_torch():
    p = mlp.init_params(0).astype(np.float64)
    x = np.random.default_rng(1).standard_normal((50, 8))
    np.testing.assert_allclose(mlp.forward(p, x), torch_forward(p, x).numpy(), rtol=1e-12, atol=1e-12)


def test_gradient_finite_differences_and_autograd():
    rng = np.random.default_rng(5)
    p = mlp.init_params(1).astype(np.float64) * 2.0
    x = rng.standard_normal((40, 8))
    t = rng.standard_normal((40, 3))
    scale = np.array([0.3, 0.5, 0.5])
    lam = 0.1
    L, g = mlp.loss_and_grad(p, x, t, scale, lam)
    # autograd with the indicator target held constant
    tp = torch.tensor(p, requires_grad=True)
    o = 0
    a = torch.tensor(x)
    for li, (i, n) in enumerate(mlp.LAYERS):
        W = tp[o:o + i * n].reshape(i, n)
        o += i * n
        b = tp[o:o + n]
        o += n
        a = a @ W + b
        if li < len(mlp.LAYERS) - 1:
            u = torch.clamp(a, -4.0, 4.0)
            a = a * (0.5 + u * (0.25 - u.abs() / 32.0))
    d = a[:, :3] - torch.tensor(t)
    e = torch.log10((d.detach().abs() * torch.tensor(scale)).max(1).values + mlp.ERR_FLOOR)
    Lt = (d * d).sum() / (3 * 40) + lam * ((a[:, 3] - e) ** 2).sum() / 40
    Lt.backward()
    assert abs(float(Lt.detach()) - L) < 1e-12 * max(1.0, abs(L))
    np.testing.assert_allclose(g, tp.grad.numpy(), rtol=1e-10, atol=1e-13)
    # central differences on sampled parameters (e is recomputed, so stay away from its kinks)
    idx = rng.choice(mlp.N_PARAMS, 40, replace=False)
    for k in idx:
        eps = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += eps
        pm[k] -= eps
        fd = (mlp.loss_and_grad(pp, x, t, scale, 0.0)[0] - mlp.loss_and_grad(pm, x, t, scale, 0.0)[0]) / (2 * eps)
        g0 = mlp.loss_and_grad(p, x, t, scale, 0.0)[1][k]
        assert abs(fd - g0) <= 1e-7 * max(1.0, abs(g0)), k


def test_rounded_forward_close_to_exact():
    p = mlp.init_params(2).astype(np.float64)
    x = np.random.default_rng(2).standard_normal((200, 8))
    a = mlp.forward(p, x)
    b = mlp.forward(p, x, round_bf16=True)
    assert np.abs(a - b).max() < 0.05 * np.abs(a).max()
    assert np.abs(a - b).max() > 0.0


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    p = rng.standard_normal(100)
    m = np.zeros(100)
    v = np.zeros(100)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.standard_normal(100)
        p, m, v = mlp.adam(p, m, v, g, step, 3e-3)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)

"""Pins of the FP64 reference of the learned correction (oracle/learned.py)
and of the oracle's extra body force.

Each pin comes from outside the code under test: published constants of the
normal distribution, torch's own GELU, autograd and Adam (CPU, float64), finite
differences, exact discrete identities and conservation.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import learned as L
from tests import inputs


def test_gelu_values_and_symmetry():
    # Phi(1) and Phi(-1), Phi(2) from tables of the standard normal CDF
    assert abs(L.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(L.gelu(-1.0) - (-0.15865525393145707)) < 1e-15
    assert abs(L.gelu(2.0) - 2 * 0.9772498680518208) < 1e-15
    z = np.linspace(-6, 6, 97)
    assert np.allclose(L.gelu(z) - L.gelu(-z), z, atol=1e-15, rtol=0)
    h = 1e-6
    fd = (L.gelu(z + h) - L.gelu(z - h)) / (2 * h)
    assert np.allclose(L.gelu_grad(z), fd, atol=1e-9, rtol=0)


def test_gelu_matches_torch_exact_gelu():
    z = inputs.normal(3, (200,), 2.0)
    ref = torch.nn.functional.gelu(torch.tensor(z, dtype=torch.float64), approximate="none")
    assert np.allclose(L.gelu(z), ref.numpy(), atol=1e-15, rtol=1e-14)


def _torch_net(p):
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}

    def f(X):
        G = lambda a: torch.nn.functional.gelu(a, approximate="none")
        h1 = G(torch.nn.functional.linear(X, t["W1"], t["b1"]))
        h2 = G(torch.nn.functional.linear(h1, t["W2"], t["b2"]))
        return torch.nn.functional.linear(h2, t["W3"], t["b3"])
    return t, f


def test_forward_and_backward_match_torch_autograd():
    p = L.init_params(54, 64, 5, seed=4)
    for k in p:
        if k[0] == "b":
            p[k] = inputs.normal(20 + int(k[1]), p[k].shape, 0.1)
    X = inputs.normal(5, (37, 54))
    T = inputs.normal(6, (37, 5))
    Y, cache = L.forward(p, X)
    g = L.backward(p, cache, Y, T)
    t, f = _torch_net(p)
    Yt = f(torch.tensor(X))
    assert np.allclose(Y, Yt.detach().numpy(), atol=1e-13, rtol=1e-12)
    lt = torch.mean((Yt - torch.tensor(T)) ** 2)
    lt.backward()
    assert abs(L.loss(Y, T) - lt.item()) < 1e-14
    for k in p:
        assert np.allclose(g[k], t[k].grad.numpy(), atol=1e-14, rtol=1e-11), k


def test_backward_matches_finite_differences():
    """Gradient check: central differences of the loss in every parameter of
    a small network."""
    p = L.init_params(6, 4, 3, seed=7)
    for k in p:
        p[k] = p[k] + inputs.normal(len(k) + 11, p[k].shape, 0.2)
    X = inputs.normal(8, (9, 6))
    T = inputs.normal(9, (9, 3))
    Y, cache = L.forward(p, X)
    g = L.flatten(L.backward(p, cache, Y, T))
    theta = L.flatten(p)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = L.loss(L.forward(L.unflatten(tp, 6, 4, 3), X)[0], T)
        lm = L.loss(L.forward(L.unflatten(tm, 6, 4, 3), X)[0], T)
        fd[i] = (lp - lm) / (2 * h)
    assert np.abs(g - fd).max() < 1e-8 * max(1.0, np.abs(g).max())


def test_adam_matches_torch():
    theta0 = inputs.normal(10, (20,))
    grads = [inputs.normal(11 + i, (20,)) for i in range(4)]
    th, m, v = theta0.copy(), np.zeros(20), np.zeros(20)
    for i, gr in enumerate(grads, start=1):
        th, m, v = L.adam(th, gr, m, v, i, lr=1e-2)
    w = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for gr in grads:
        opt.zero_grad()
        w.grad = torch.tensor(gr, dtype=torch.float64)
        opt.step()
    assert np.allclose(th, w.detach().numpy(), atol=1e-15, rtol=1e-13)


def test_restriction_invariants():
    m = 4
    f = inputs.normal(12, (3, 16, 24))
    r = L.restrict(f, m)
    assert r.shape == (3, 4, 6)
    # total conserved up to the area factor
    assert np.allclose(r.sum(axis=(1, 2)) * m * m, f.sum(axis=(1, 2)), rtol=1e-13)
    # constants are kept
    assert np.allclose(L.restrict(np.full((8, 8), 2.5), m), 2.5, atol=1e-15)
    # a function linear in x and y (away from the periodic seam) is sampled at
    # the coarse node centre
    y, x = np.mgrid[0:32, 0:32].astype(float)
    lin = 0.3 * x - 0.7 * y + 1.0
    rl = L.restrict(lin, m)
    Y, X = np.mgrid[1:7, 1:7]
    assert np.allclose(rl[1:7, 1:7], 0.3 * (m * X) - 0.7 * (m * Y) + 1.0, atol=1e-13)


def test_features_layout():
    ny, nx = 3, 4
    obs = np.zeros((10, ny, nx))
    for f in range(10):
        obs[f] = 1000 * f + 10 * np.arange(ny)[:, None] + np.arange(nx)[None, :]
    X = L.features(obs)
    assert X.shape == (12, 54)
    # node (y=0, x=0): stencil position (dy=-1, dx=-1) is the periodic corner (2, 3)
    assert X[0, 0] == 0 + 10 * 2 + 3           # rho at (2, 3)
    assert X[0, 5] == 6000 + 10 * 2 + 3        # Cyy at (2, 3)
    # centre (s = 4) of node (1, 2), field Ux
    assert X[1 * nx + 2, 6 * 4 + 1] == 1000 + 10 * 1 + 2
    # (dy=+1, dx=+1) of node (2, 3) wraps to (0, 0), field Cxy (index 5 -> pos 4)
    assert X[2 * nx + 3, 6 * 8 + 4] == 5000


def test_source_divergence_identity_and_momentum():
    ny, nx = 16, 12
    ky, kx = 2 * math.pi * 2 / ny, 2 * math.pi * 3 / nx
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    corr = np.zeros((ny * nx, 5))
    corr[:, 0] = 1e-3
    corr[:, 2] = np.sin(kx * x).ravel()      # tau_xx
    corr[:, 3] = np.cos(ky * y).ravel()      # tau_xy
    corr[:, 1] = np.cos(kx * x).ravel() * 1e-3 + 2e-4  # a mean and a mode
    F = L.source(corr, ny, nx)
    # exact discrete identities of the central difference; the uniform
    # momentum correction is removed, its fluctuating part kept
    assert np.allclose(F[0], math.sin(kx) * np.cos(kx * x) - math.sin(ky) * np.sin(ky * y),
                       atol=1e-14)
    assert np.allclose(F[1], 1e-3 * np.cos(kx * x), atol=1e-14)
    # the source injects no net momentum
    assert abs(F[0].sum()) < 1e-12 and abs(F[1].sum()) < 1e-12


def test_oracle_source_injects_its_momentum():
    o = oracle.OracleSim(8, 8, nq=4)
    o.rest()
    F = np.stack([inputs.normal(13, (8, 8), 1e-5), inputs.normal(14, (8, 8), 1e-5)])
    o.set_source(F)
    d0 = o.diagnostics()
    o.step(3)
    d1 = o.diagnostics()
    # forcing of one period sums to zero; the source adds sum(F) per step
    assert abs((d1["mom_x"] - d0["mom_x"]) - 3 * F[0].sum()) < 1e-14
    assert abs((d1["mom_y"] - d0["mom_y"]) - 3 * F[1].sum()) < 1e-14
    assert abs(d1["mass_S"] - d0["mass_S"]) < 1e-13
    o.set_source(None)
    o.step(1)
    d2 = o.diagnostics()
    assert abs(d2["mom_x"] - d1["mom_x"]) < 1e-14

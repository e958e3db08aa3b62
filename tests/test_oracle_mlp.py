"""Pins of the warm-start network oracle and its inputs.

The forward pass and the Adam step are compared with PyTorch's CPU float64
routines (torch.nn.functional.linear / silu, torch.optim.Adam); the gradient
with central finite differences; the neighbour list with a brute-force scan
and the graphene shell distances.
"""
import math

import numpy as np
import pytest
import torch

from oracle import features as ft
from oracle import mlp
from paper_2111_06704_amd import workloads as wl


def _theta(seed=0):
    rng = np.random.default_rng(seed)
    th = mlp.init_params(rng)
    th[mlp.NIN * mlp.NH: mlp.NIN * mlp.NH + mlp.NH] = rng.standard_normal(mlp.NH) * 0.1   # b1
    return th


def test_forward_matches_torch():
    th = _theta(1)
    X = np.random.default_rng(2).standard_normal((37, mlp.NIN))
    p = mlp.unpack(th)
    Xt = torch.tensor(X)
    h1 = torch.nn.functional.silu(torch.nn.functional.linear(Xt, torch.tensor(p["W1"]).T, torch.tensor(p["b1"])))
    h2 = torch.nn.functional.silu(torch.nn.functional.linear(h1, torch.tensor(p["W2"]).T, torch.tensor(p["b2"])))
    y = h2 @ torch.tensor(p["W3"]) + torch.tensor(p["b3"])
    assert np.allclose(mlp.forward(th, X), y.numpy(), rtol=1e-13, atol=1e-13)


def test_gradient_central_differences():
    th = _theta(3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((11, mlp.NIN))
    t = rng.standard_normal(11)
    loss, g = mlp.loss_grad(th, X, t)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, mlp.NIN * mlp.NH]])
    h = 1e-6
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (np.mean((mlp.forward(tp, X) - t) ** 2) - np.mean((mlp.forward(tm, X) - t) ** 2)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k
    assert abs(loss - np.mean((mlp.forward(th, X) - t) ** 2)) < 1e-15


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    th = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    w = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        th, m, v = mlp.adam_step(th, m, v, g, step, 3e-3)
        opt.zero_grad()
        w.grad = torch.tensor(g)
        opt.step()
    assert np.allclose(th, w.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_neighbour_list_graphene():
    geo = wl.geometry(1)
    nbr, dist = ft.neighbours(geo.pos, geo.box)
    assert np.array_equal(nbr, ft.neighbours_brute(geo.pos, geo.box))
    R = wl.BOND
    shells = np.array([R] * 3 + [math.sqrt(3) * R] * 6 + [2 * R] * 3)
    assert np.allclose(dist, shells[None, :], atol=1e-9)
    # in-plane neighbours only (sheets are 40 A apart)
    assert np.all(geo.electrode[nbr] == geo.electrode[:, None])


def test_neighbour_list_graphite_jittered():
    geo = wl.jitter(wl.geometry(2), 0.01, 7)
    sub = np.arange(0, geo.n, 37)
    nbr, _ = ft.neighbours(geo.pos, geo.box)
    full = ft.neighbours_brute(geo.pos, geo.box)
    assert np.array_equal(nbr[sub], full[sub])


def test_features_layout_and_gauge():
    geo = wl.geometry(1)
    nbr, dist = ft.neighbours(geo.pos, geo.box)
    rng = np.random.default_rng(6)
    b = rng.standard_normal((2, geo.n))
    X = ft.features(b, nbr, dist, geo.layer, geo.n_layers, 0.5, 2.0)
    assert X.shape == (2 * geo.n, 26)
    i = 17
    row = X[geo.n + i]
    bc = (b[1] - b[1].mean()) / 0.5
    assert row[0] == bc[i] and row[1] == geo.layer[i] / (geo.n_layers - 1)
    assert np.array_equal(row[2:14], bc[nbr[i]]) and np.allclose(row[14:], dist[i] / 2.0)
    # a uniform shift of b (gauge, Eq. 29) leaves the inputs unchanged
    X2 = ft.features(b + 3.0, nbr, dist, geo.layer, geo.n_layers, 0.5, 2.0)
    assert np.allclose(X, X2, atol=1e-13)

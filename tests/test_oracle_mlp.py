"""Pins of the oracle network (closed forms, finite differences, the Adam
update rule) and of the oracle projection (functions in the span, the normal
equations)."""
import math

import numpy as np
import pytest

import rfm_workloads as W
from oracle import mlp as M
from oracle import rfm as O


def test_forward_closed_form_one_unit():
    # y = w2 tanh(w1 x + b1) + b2
    ds = M.dims(1, 1, 1, 1)
    p = np.array([0.7, -0.2, 1.3, 0.4])
    x = np.array([[0.5], [-1.0]])
    y, _ = M.forward(p, ds, x)
    ref = 1.3 * np.tanh(0.7 * x - 0.2) + 0.4
    assert np.allclose(y, ref, rtol=0, atol=1e-15)


def test_gradient_by_central_differences():
    ds = M.dims(3, 5, 2, 2)
    p = W.mlp_params(3, 5, 2, 2, seed=3).astype(np.float64)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(7, 3))
    Y = rng.normal(size=(7, 2))
    L, g = M.loss_grad(p, ds, X, Y)
    h = 1e-6
    fd = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss_grad(p + e, ds, X, Y)[0] - M.loss_grad(p - e, ds, X, Y)[0]) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-8 * np.linalg.norm(fd)
    assert abs(L - np.mean((M.forward(p, ds, X)[0] - Y) ** 2)) < 1e-15


def test_bf16_operands_change_little():
    ds = M.dims(6, 32, 3, 2)
    p = W.mlp_params(6, 32, 3, 2, seed=5).astype(np.float64)
    X = np.random.default_rng(6).uniform(0, 1, size=(50, 6))
    y0, _ = M.forward(p, ds, X)
    y1, _ = M.forward(p, ds, X, bf16=True)
    rel = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
    assert 1e-5 < rel < 3e-2          # rounding is visible but at the BF16 level (2^-9 per operand)


def test_adam_first_steps():
    # step 1 from zero moments: m_hat = g, v_hat = g^2, so the move is -lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = M.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    # step 2 with the same gradient: moments are bias-corrected back to g and g^2
    p2, _, _ = M.adam(p, m, v, g, 2, lr=0.01)
    assert np.allclose(p2 - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    # hand computation of step 2 with a different gradient
    g2 = np.array([1.0, 1.0, 1.0, 1.0])
    p3, m3, v3 = M.adam(p, m, v, g2, 2, lr=0.01, b1=0.9, b2=0.999)
    mm = 0.9 * 0.1 * g + 0.1 * g2
    vv = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    step = -0.01 * (mm / (1 - 0.81)) / (np.sqrt(vv / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(p3 - p, step, rtol=1e-12)


def _small_gs():
    return W.gray_scott_member(0.04, 0.06, 0.5, nsub=(2, 1, 1), J=20, q=4, test_per_dim=2)


def test_projection_reproduces_functions_in_the_span():
    prob = _small_gs()
    Phi = O.feature_matrix_pde(prob)
    u_true = np.random.default_rng(7).normal(size=prob.n)
    f = Phi @ u_true                     # [npde * ncomp] in (group, comp, point) order
    x, _ = O.pde_points(prob)
    vals = np.zeros((len(x), prob.ncomp))
    base = 0
    k0 = 0
    for g in prob.groups:
        if g.kind != W.KIND_PDE:
            continue
        n = len(g.x)
        for k in range(prob.ncomp):
            vals[base:base + n, k] = f[k0:k0 + n]
            k0 += n
        base += n
    u = O.project(prob, vals)
    assert np.linalg.norm(Phi @ u - f) <= 1e-8 * np.linalg.norm(f)


def test_projection_normal_equations():
    prob = _small_gs()
    x, _ = O.pde_points(prob)
    vals = np.stack([np.sin(3 * x[:, 0]) + x[:, 1], np.cos(2 * x[:, 2])], axis=1)
    u = O.project(prob, vals)
    Phi = O.feature_matrix_pde(prob)
    D = O.row_scale(Phi)
    f = []
    base = 0
    for g in prob.groups:
        if g.kind != W.KIND_PDE:
            continue
        n = len(g.x)
        for k in range(prob.ncomp):
            f.append(vals[base:base + n, k])
        base += n
    f = np.concatenate(f)
    r = D * (Phi @ u - f)
    # the weighted residual is orthogonal to the range of D Phi
    assert np.linalg.norm((D[:, None] * Phi).T @ r) <= 1e-7 * np.linalg.norm(D[:, None] * Phi) * np.linalg.norm(D * f)

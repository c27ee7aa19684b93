"""Pins of the oracle's coupling flow, its loss gradient and Adam."""
import math

import numpy as np
import pytest

from oracle import flow
from oracle.integrands import gauss, gauss_integral
from synth import he_init_segments


def random_theta(dim, L, K, H, seed, out_scale=1.0):
    rng = np.random.default_rng(seed)
    th = he_init_segments(flow.init_segments(dim, L, K, H), seed).astype(np.float64)
    # give the zero-initialised output layers non-trivial values
    off = 0
    for sh in flow.layer_shapes(dim, L, K, H):
        sz = sh["sizes"]
        o3 = off + sum(sz[:4])
        th[o3:o3 + sz[4] + sz[5]] = rng.normal(0, out_scale, sz[4] + sz[5])
        off += sum(sz)
    return th


def test_parameter_counts():
    assert flow.n_params(8, 4, 32, 64) == 51200
    assert flow.n_params(3, 4, 32, 64) == 29760
    assert flow.masks(3, 4) == [([0, 2], [1]), ([1], [0, 2]), ([0, 1], [2]), ([2], [0, 1])]
    for A, B in flow.masks(8, 4):
        assert sorted(A + B) == list(range(8)) and len(B) == 4


def test_zero_output_layer_is_identity():
    th = he_init_segments(flow.init_segments(3, 4, 32, 64), 0).astype(np.float64)
    y = np.random.default_rng(0).uniform(size=(500, 3))
    u, logq = flow.density(th, y, 3, 4, 32, 64)
    assert np.allclose(u, y, rtol=0, atol=1e-15)
    assert np.allclose(logq, 0.0, atol=1e-14)
    y2, lq2 = flow.sample(th, y, 3, 4, 32, 64)
    assert np.allclose(y2, y, rtol=0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3, 8])
def test_sample_and_density_invert_each_other(dim):
    th = random_theta(dim, 4, 32, 16, seed=dim)
    u = np.random.default_rng(1).uniform(size=(2000, dim))
    y, lq = flow.sample(th, u, dim, 4, 32, 16)
    assert np.all((y >= 0) & (y <= 1))
    u2, lq2 = flow.density(th, y, dim, 4, 32, 16)
    assert np.max(np.abs(u2 - u)) < 1e-12
    assert np.max(np.abs(lq2 - lq)) < 1e-9


def test_single_layer_density_normalised_along_transformed_dim():
    # one layer, A = {0}, B = {1}: for fixed y0 the density in y1 is
    # piecewise constant on the K bins, so a bin-aligned midpoint sum is exact.
    th = random_theta(2, 1, 8, 16, seed=3, out_scale=2.0)
    for y0 in (0.1, 0.55, 0.93):
        m = 8 * 16
        y1 = (np.arange(m) + 0.5) / m
        y = np.column_stack([np.full(m, y0), y1])
        _, logq = flow.density(th, y, 2, 1, 8, 16)
        assert np.mean(np.exp(logq)) == pytest.approx(1.0, rel=1e-13)


def test_density_integrates_to_one_monte_carlo():
    th = random_theta(3, 4, 32, 16, seed=5, out_scale=0.7)
    y = np.random.default_rng(2).uniform(size=(200000, 3))
    _, logq = flow.density(th, y, 3, 4, 32, 16)
    q = np.exp(logq)
    assert abs(q.mean() - 1.0) < 5 * q.std() / math.sqrt(len(q))


def test_gradient_matches_finite_differences():
    dim, L, K, H = 3, 4, 4, 8
    th = random_theta(dim, L, K, H, seed=7, out_scale=0.8)
    rng = np.random.default_rng(3)
    y = rng.uniform(size=(64, dim))
    g = gauss(y, 0.5, 0.2) + 0.1
    _, grad, _ = flow.loss_and_grad(th, y, g, dim, L, K, H)
    idx = rng.choice(th.size, 80, replace=False)
    h = 1e-5  # rounding error of the difference ~ eps |L| / h ~ 1e-10
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (flow.loss(tp, y, g, dim, L, K, H) - flow.loss(tm, y, g, dim, L, K, H)) / (2 * h)
        assert grad[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_constant_gradient_and_quadratic():
    th, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    g = np.array([2.0, -0.5, 1e-3])
    for t in range(1, 6):
        new, m, v = flow.adam_step(th, m, v, g, t, lr=0.01)
        assert np.allclose(new - th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        th = new
    x, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 3001):
        x, m, v = flow.adam_step(x, m, v, 2 * (x - 3.0), t, lr=0.05)
    assert x[0] == pytest.approx(3.0, abs=1e-3)


def test_weights_g_over_q_are_unbiased_for_random_flow():
    dim = 2
    th = random_theta(dim, 4, 32, 16, seed=11, out_scale=0.5)
    u = np.random.default_rng(4).uniform(size=(200000, dim))
    y, logq = flow.sample(th, u, dim, 4, 32, 16)
    w = gauss(y, 0.4, 0.2) * np.exp(-logq)
    I = gauss_integral(dim, 0.4, 0.2)
    assert abs(w.mean() - I) < 4 * w.std() / math.sqrt(len(w))


def test_training_reduces_variance():
    # a few Adam steps on the normalised second moment lower it, and the
    # trained flow's g/q has a smaller variance than uniform sampling.
    dim, L, K, H = 2, 4, 16, 16
    th = he_init_segments(flow.init_segments(dim, L, K, H), 1).astype(np.float64)
    rng = np.random.default_rng(5)
    f = lambda x: gauss(x, 0.3, 0.1)
    m, v = np.zeros_like(th), np.zeros_like(th)
    first = None
    for t in range(1, 61):
        y = rng.uniform(size=(4000, dim))
        Lv, grad, _ = flow.loss_and_grad(th, y, f(y), dim, L, K, H)
        first = Lv if first is None else first
        th, m, v = flow.adam_step(th, m, v, grad, t, lr=1e-2)
    u = rng.uniform(size=(50000, dim))
    y, logq = flow.sample(th, u, dim, L, K, H)
    w = f(y) * np.exp(-logq)
    w0 = f(u)
    assert w.var() < 0.5 * w0.var()
    assert Lv < 0.7 * first


def test_gradient_magnitudes_bound_the_per_sample_terms():
    """The magnitude of each gradient element (the gradient formula on
    absolute values) bounds the sum over samples of |per-sample gradient|,
    which bounds |gradient|.  The loss is sum_s g_s^2 q_s^-1 / (n mean g^2)
    with mean g^2 fixed by the batch, so sample s's share of the gradient
    is g_s^2 / (n mean g^2) times the gradient of the one-sample loss q_s^-1."""
    dim, L, K, H = 3, 4, 8, 8
    th = random_theta(dim, L, K, H, seed=12, out_scale=0.8)
    rng = np.random.default_rng(6)
    y = rng.uniform(size=(24, dim))
    g = gauss(y, 0.5, 0.2) + 0.1
    _, grad, _, mag = flow.loss_and_grad(th, y, g, dim, L, K, H, magnitudes=True)
    _, grad0, _ = flow.loss_and_grad(th, y, g, dim, L, K, H)
    assert np.array_equal(grad, grad0)
    m2 = np.mean(g ** 2)
    per = np.zeros_like(grad)
    for s in range(len(y)):
        _, gs, _ = flow.loss_and_grad(th, y[s:s + 1], g[s:s + 1], dim, L, K, H)
        per += np.abs(gs) * g[s] ** 2 / (len(y) * m2)
    assert np.all(per <= mag * (1 + 1e-12) + 1e-300)
    assert np.all(np.abs(grad) <= per * (1 + 1e-12) + 1e-300)
    # the magnitude is not a loose multiple of the gradient: some elements
    # (no cancellation) meet it, and it is finite and non-zero where the
    # gradient is
    nz = np.abs(grad) > 0
    assert np.all(mag[nz] > 0) and np.all(np.isfinite(mag))
    assert np.max(np.abs(grad[nz]) / mag[nz]) > 0.99

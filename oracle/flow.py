"""Piecewise-linear coupling flow, variance loss, gradients, Adam (oracle).

TEST INFRASTRUCTURE.  The thesis contains no normalizing flow; it gives the
importance-sampling estimator and its variance (Monte Carlo chapter), the
dense layer y = phi(W x + b) and the activation table (deep-learning
chapter), the training loop and the Adam equations with beta1 = 0.9,
beta2 = 0.999, eps = 1e-8 (optimiser section).  The coupling transform is
the piecewise-linear one of Mueller et al., "Neural importance sampling",
2019; the readings used:

  * d >= 2 dimensions, L coupling layers.  Layer l transforms the dims B_l
    conditioned on the others A_l, with  k = (l // 2) mod ceil(log2 d),
    B_l = { j : bit k of j == (1 if l even else 0) }.
  * Each layer's network: |A| -> H -> H -> |B| K, ReLU on the hidden
    layers, softmax over the K logits of each transformed dim giving bin
    probabilities Q_0..Q_{K-1}.  Parameters per layer, flat and in this
    order: W1 [H][|A|], b1 [H], W2 [H][H], b2 [H], W3 [|B| K][H], b3 [|B| K]
    (row-major, output index first); the logits of B-dim jb are rows
    jb K .. jb K + K - 1.
  * Density direction (y -> u), layers l = 0 .. L-1 in order: for j in B,
    b = min(floor(K z_j), K - 1), alpha = K z_j - b,
    z_j <- sum_{k<b} Q_k + alpha Q_b, and log q += ln(K Q_b).
  * Sampling direction (u -> y), layers l = L-1 .. 0: for j in B, b with
    C_b <= v < C_{b+1} (C the cumulative Q), z_j <- (b + (v - C_b)/Q_b)/K,
    and log q += ln(K Q_b).  It inverts the density direction exactly, and
    q(y) = prod over layers and B dims of K Q_b is the sampling density.
  * Training data are uniform points y of the VEGAS unit cube with
    g(y) = f(G(y)) J_G(y); the loss is the second moment of g/q under
    y ~ U, normalised by the batch mean of g^2 (a constant per batch):
        L = mean(g^2 / q) / mean(g^2),
    whose minimum is at q proportional to |g| (zero-variance importance
    sampling), and dL/dlog q_i = -(g_i^2/q_i) / (n mean(g^2)).

Pins: tests/test_oracle_flow.py -- sampling and density directions invert
each other; q integrates to 1 (lattice sum); zero output weights give the
identity map with q = 1; analytic gradients match central finite
differences; Adam on a constant gradient g moves every step by exactly
lr g/(|g| + eps) (bias corrections cancel), and it converges on a
one-dimensional quadratic; unbiasedness of g/q for trained and random
weights.
"""
import math

import numpy as np


def n_bits(dim):
    return max(1, int(math.ceil(math.log2(dim))))


def masks(dim, n_layers):
    """List of (A, B) index lists per layer."""
    out = []
    nb = n_bits(dim)
    for layer in range(n_layers):
        k = (layer // 2) % nb
        par = 1 if layer % 2 == 0 else 0
        B = [j for j in range(dim) if ((j >> k) & 1) == par]
        A = [j for j in range(dim) if ((j >> k) & 1) != par]
        if not A or not B:
            raise ValueError("dimension too small for the coupling masks")
        out.append((A, B))
    return out


def layer_shapes(dim, n_layers, n_bins, hidden):
    shapes = []
    for A, B in masks(dim, n_layers):
        a, b = len(A), len(B)
        shapes.append(dict(A=A, B=B, sizes=[hidden * a, hidden, hidden * hidden, hidden,
                                                b * n_bins * hidden, b * n_bins]))
    return shapes


def init_segments(dim, n_layers, n_bins, hidden):
    """Segment list (kind, fan_in, size) for synth.he_init_segments."""
    segs = []
    for sh in layer_shapes(dim, n_layers, n_bins, hidden):
        a = len(sh["A"])
        b = len(sh["B"])
        segs += [("w", a, hidden * a), ("b", a, hidden), ("w", hidden, hidden * hidden),
                 ("b", hidden, hidden), ("z", hidden, b * n_bins * hidden), ("z", hidden, b * n_bins)]
    return segs


def n_params(dim, n_layers, n_bins, hidden):
    return sum(sum(sh["sizes"]) for sh in layer_shapes(dim, n_layers, n_bins, hidden))


def unpack(theta, dim, n_layers, n_bins, hidden):
    theta = np.asarray(theta, dtype=np.float64)
    layers = []
    off = 0
    for sh in layer_shapes(dim, n_layers, n_bins, hidden):
        a, b = len(sh["A"]), len(sh["B"])
        p = {}
        for name, shape in (("W1", (hidden, a)), ("b1", (hidden,)), ("W2", (hidden, hidden)),
                            ("b2", (hidden,)), ("W3", (b * n_bins, hidden)), ("b3", (b * n_bins,))):
            size = int(np.prod(shape))
            p[name] = theta[off:off + size].reshape(shape)
            off += size
        p["A"], p["B"] = sh["A"], sh["B"]
        layers.append(p)
    assert off == theta.size
    return layers


def _mlp(p, zA, n_bins):
    pre1 = zA @ p["W1"].T + p["b1"]
    h1 = np.maximum(pre1, 0.0)
    pre2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(pre2, 0.0)
    logits = h2 @ p["W3"].T + p["b3"]
    n = zA.shape[0]
    lg = logits.reshape(n, len(p["B"]), n_bins)
    lg = lg - lg.max(axis=2, keepdims=True)
    e = np.exp(lg)
    Q = e / e.sum(axis=2, keepdims=True)
    return dict(pre1=pre1, h1=h1, pre2=pre2, h2=h2, Q=Q)


def density(theta, y, dim, n_layers, n_bins, hidden, keep=False):
    """Density direction: returns (u, log q) [and per-layer caches]."""
    layers = unpack(theta, dim, n_layers, n_bins, hidden)
    z = np.array(y, dtype=np.float64, copy=True)
    n = z.shape[0]
    logq = np.zeros(n)
    caches = []
    for p in layers:
        A, B = p["A"], p["B"]
        m = _mlp(p, z[:, A], n_bins)
        Q = m["Q"]
        cum = np.concatenate([np.zeros((n, len(B), 1)), np.cumsum(Q, axis=2)], axis=2)
        zin = z.copy()
        bins = np.empty((n, len(B)), dtype=np.int64)
        alphas = np.empty((n, len(B)))
        for jb, j in enumerate(B):
            t = n_bins * z[:, j]
            b = np.minimum(np.floor(t).astype(np.int64), n_bins - 1)
            al = t - b
            qb = Q[np.arange(n), jb, b]
            z[:, j] = cum[np.arange(n), jb, b] + al * qb
            logq += np.log(n_bins * qb)
            bins[:, jb] = b
            alphas[:, jb] = al
        if keep:
            caches.append(dict(zin=zin, m=m, bins=bins, alphas=alphas))
    if keep:
        return z, logq, caches
    return z, logq


def sample(theta, u, dim, n_layers, n_bins, hidden):
    """Sampling direction: returns (y, log q)."""
    layers = unpack(theta, dim, n_layers, n_bins, hidden)
    z = np.array(u, dtype=np.float64, copy=True)
    n = z.shape[0]
    logq = np.zeros(n)
    for p in reversed(layers):
        A, B = p["A"], p["B"]
        Q = _mlp(p, z[:, A], n_bins)["Q"]
        cum = np.cumsum(Q, axis=2)
        for jb, j in enumerate(B):
            v = z[:, j]
            # b = number of interior cumulative values C_1..C_{K-1} that are <= v
            b = np.sum(cum[:, jb, :n_bins - 1] <= v[:, None], axis=1)
            b = np.minimum(b, n_bins - 1)
            cb = np.where(b > 0, cum[np.arange(n), jb, np.maximum(b - 1, 0)], 0.0)
            qb = Q[np.arange(n), jb, b]
            z[:, j] = (b + (v - cb) / qb) / n_bins
            logq += np.log(n_bins * qb)
    return z, logq


def loss(theta, y, g, dim, n_layers, n_bins, hidden):
    _, logq = density(theta, y, dim, n_layers, n_bins, hidden)
    g2 = np.asarray(g, dtype=np.float64) ** 2
    return float(np.mean(g2 * np.exp(-logq)) / np.mean(g2))


def loss_and_grad(theta, y, g, dim, n_layers, n_bins, hidden):
    """Return (L, dL/dtheta (flat, FP64), log q)."""
    y = np.asarray(y, dtype=np.float64)
    g2 = np.asarray(g, dtype=np.float64) ** 2
    n = y.shape[0]
    layers = unpack(theta, dim, n_layers, n_bins, hidden)
    _, logq, caches = density(theta, y, dim, n_layers, n_bins, hidden, keep=True)
    ratio = g2 * np.exp(-logq)
    m2 = np.mean(g2)
    L = float(np.mean(ratio) / m2)
    dlogq = -ratio / (n * m2)           # dL/dlog q_i (shared by all layers)
    dz = np.zeros_like(y)               # dL/dz at the output (u): zero
    grads = []
    for p, c in zip(reversed(layers), reversed(caches)):
        A, B = p["A"], p["B"]
        m = c["m"]
        Q = m["Q"]
        bins, alphas = c["bins"], c["alphas"]
        dQ = np.zeros_like(Q)
        dz_in = dz.copy()
        rows = np.arange(n)
        for jb, j in enumerate(B):
            b = bins[:, jb]
            al = alphas[:, jb]
            gz = dz[:, j]                 # dL/dz'_j
            # z'_j = sum_{k<b} Q_k + alpha Q_b ;  ld = ln K + ln Q_b
            mask_lt = np.arange(n_bins)[None, :] < b[:, None]
            dQ[:, jb, :] += gz[:, None] * mask_lt
            qb = Q[rows, jb, b]
            dQ[rows, jb, b] += gz * al + dlogq / qb
            dz_in[:, j] = gz * n_bins * qb  # dz'_j/dz_j = K Q_b
        # softmax backward
        dlog = Q * (dQ - np.sum(Q * dQ, axis=2, keepdims=True))
        dlog = dlog.reshape(n, -1)
        gW3 = dlog.T @ m["h2"]
        gb3 = dlog.sum(axis=0)
        dh2 = dlog @ p["W3"]
        dpre2 = dh2 * (m["pre2"] > 0)
        gW2 = dpre2.T @ m["h1"]
        gb2 = dpre2.sum(axis=0)
        dh1 = dpre2 @ p["W2"]
        dpre1 = dh1 * (m["pre1"] > 0)
        zA = c["zin"][:, A]
        gW1 = dpre1.T @ zA
        gb1 = dpre1.sum(axis=0)
        dzA = dpre1 @ p["W1"]
        dz_in[:, A] += dzA
        dz = dz_in
        grads.append([gW1, gb1, gW2, gb2, gW3, gb3])
    flat = np.concatenate([np.concatenate([t.ravel() for t in gl]) for gl in reversed(grads)])
    return L, flat, logq


def adam_step(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (thesis optimiser section), step number t >= 1.

    m_t = b1 m + (1-b1) g;  v_t = b2 v + (1-b2) g^2;
    mhat = m_t/(1-b1^t);  vhat = v_t/(1-b2^t);
    theta_t = theta - lr mhat/(sqrt(vhat) + eps).
    """
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v

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

Two optional arguments serve the parity tests and leave the arithmetic
above unchanged when absent: an `operand` hook that maps each input of a
matrix product to the value a reduced-precision product takes (the
spec fixes BF16 operands with FP32 accumulation for the networks),
and gradient magnitudes (the gradient formula on absolute values), the
scale of the rounding error of any evaluation order.

Pins: tests/test_oracle_flow.py -- sampling and density directions invert
each other; q integrates to 1 (lattice sum); zero output weights give the
identity map with q = 1; analytic gradients match central finite
differences; the magnitudes bound the per-sample gradient terms (brute
force over samples); Adam on a constant gradient g moves every step by
exactly lr g/(|g| + eps) (bias corrections cancel), and it converges on a
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


def _same(a, mag=None):
    return a


def _mlp(p, zA, n_bins, operand=_same):
    """The layer's network.  `operand(a, mag)` maps each input of a matrix
    product (the layer input and the two hidden activations) to the value
    the product takes, given the sum of the magnitudes of the terms that
    formed it (mag); the identity (default) is the plain FP64 network, and
    tests pass a model of reduced-precision operands."""
    a0 = operand(zA, np.abs(zA))
    pre1 = a0 @ p["W1"].T + p["b1"]
    h1 = np.maximum(pre1, 0.0)
    a1 = h1 if operand is _same else operand(h1, np.abs(a0) @ np.abs(p["W1"]).T + np.abs(p["b1"]))
    pre2 = a1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(pre2, 0.0)
    a2 = h2 if operand is _same else operand(h2, np.abs(a1) @ np.abs(p["W2"]).T + np.abs(p["b2"]))
    logits = a2 @ p["W3"].T + p["b3"]
    n = zA.shape[0]
    lg = logits.reshape(n, len(p["B"]), n_bins)
    lg = lg - lg.max(axis=2, keepdims=True)
    e = np.exp(lg)
    Q = e / e.sum(axis=2, keepdims=True)
    return dict(pre1=pre1, h1=h1, pre2=pre2, h2=h2, Q=Q, a0=a0, a1=a1, a2=a2)


def density(theta, y, dim, n_layers, n_bins, hidden, keep=False, operand=_same):
    """Density direction: returns (u, log q) [and per-layer caches]."""
    layers = unpack(theta, dim, n_layers, n_bins, hidden)
    z = np.array(y, dtype=np.float64, copy=True)
    n = z.shape[0]
    logq = np.zeros(n)
    caches = []
    for p in layers:
        A, B = p["A"], p["B"]
        m = _mlp(p, z[:, A], n_bins, operand)
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


def sample(theta, u, dim, n_layers, n_bins, hidden, operand=_same):
    """Sampling direction: returns (y, log q)."""
    layers = unpack(theta, dim, n_layers, n_bins, hidden)
    z = np.array(u, dtype=np.float64, copy=True)
    n = z.shape[0]
    logq = np.zeros(n)
    for p in reversed(layers):
        A, B = p["A"], p["B"]
        Q = _mlp(p, z[:, A], n_bins, operand)["Q"]
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


def loss_and_grad(theta, y, g, dim, n_layers, n_bins, hidden, operand=_same, magnitudes=False):
    """Return (L, dL/dtheta (flat, FP64), log q) [, magnitudes].

    `operand(a, mag)` maps every input of a matrix product, forward (layer
    input, hidden activations) and backward (the deltas that meet the
    weights and the activations), to the value the product takes, given the
    sum of the magnitudes of the terms that formed it; the identity
    (default) is plain FP64.

    magnitudes=True also returns, per parameter, the same gradient formula
    evaluated on magnitudes: every product of a delta and an activation
    taken as the product of their magnitudes, every sum or difference (the
    hidden units' pre-activations, the softmax backward's dQ_k - sum Q dQ,
    the deltas' dot products with the weights, the sums over samples) as
    the sum of the absolute values of its terms.  It bounds |dL/dtheta_p| from above and sets the scale of
    the rounding error of any evaluation order of the gradient (the
    running-error bound of a sum); where no cancellation occurs it equals
    |dL/dtheta_p|.
    """
    y = np.asarray(y, dtype=np.float64)
    g2 = np.asarray(g, dtype=np.float64) ** 2
    n = y.shape[0]
    layers = unpack(theta, dim, n_layers, n_bins, hidden)
    _, logq, caches = density(theta, y, dim, n_layers, n_bins, hidden, keep=True, operand=operand)
    ratio = g2 * np.exp(-logq)
    m2 = np.mean(g2)
    L = float(np.mean(ratio) / m2)
    dlogq = -ratio / (n * m2)           # dL/dlog q_i (shared by all layers)
    dz = np.zeros_like(y)               # dL/dz at the output (u): zero
    mz = np.zeros_like(y)               # its magnitude
    grads, mags = [], []
    for p, c in zip(reversed(layers), reversed(caches)):
        A, B = p["A"], p["B"]
        m = c["m"]
        Q = m["Q"]
        bins, alphas = c["bins"], c["alphas"]
        dQ = np.zeros_like(Q)
        mQ = np.zeros_like(Q)
        dz_in = dz.copy()
        mz_in = mz.copy()
        rows = np.arange(n)
        for jb, j in enumerate(B):
            b = bins[:, jb]
            al = alphas[:, jb]
            gz = dz[:, j]                 # dL/dz'_j
            # z'_j = sum_{k<b} Q_k + alpha Q_b ;  ld = ln K + ln Q_b
            mask_lt = np.arange(n_bins)[None, :] < b[:, None]
            dQ[:, jb, :] += gz[:, None] * mask_lt
            mQ[:, jb, :] += mz[:, j][:, None] * mask_lt
            qb = Q[rows, jb, b]
            dQ[rows, jb, b] += gz * al + dlogq / qb
            mQ[rows, jb, b] += mz[:, j] * al + np.abs(dlogq) / qb
            dz_in[:, j] = gz * n_bins * qb  # dz'_j/dz_j = K Q_b
            mz_in[:, j] = mz[:, j] * n_bins * qb
        # softmax backward
        dlog = Q * (dQ - np.sum(Q * dQ, axis=2, keepdims=True))
        dlog = dlog.reshape(n, -1)
        mlog = (Q * (mQ + np.sum(Q * mQ, axis=2, keepdims=True))).reshape(n, -1)
        if operand is _same:
            o3 = dlog
        else:
            aQ = np.abs(dQ)
            o3 = operand(dlog, (Q * (aQ + np.sum(Q * aQ, axis=2, keepdims=True))).reshape(n, -1))
        gW3 = o3.T @ m["a2"]
        gb3 = o3.sum(axis=0)
        dh2 = o3 @ p["W3"]
        dpre2 = dh2 * (m["pre2"] > 0)
        o2 = dpre2 if operand is _same else operand(dpre2, (np.abs(o3) @ np.abs(p["W3"])) * (m["pre2"] > 0))
        gW2 = o2.T @ m["a1"]
        gb2 = o2.sum(axis=0)
        dh1 = o2 @ p["W2"]
        dpre1 = dh1 * (m["pre1"] > 0)
        o1 = dpre1 if operand is _same else operand(dpre1, (np.abs(o2) @ np.abs(p["W2"])) * (m["pre1"] > 0))
        gW1 = o1.T @ m["a0"]
        gb1 = o1.sum(axis=0)
        dzA = o1 @ p["W1"]
        dz_in[:, A] += dzA
        dz = dz_in
        grads.append([gW1, gb1, gW2, gb2, gW3, gb3])
        if magnitudes:
            # activations as sums of magnitudes too (a hidden unit just above
            # zero is a cancellation of its pre-activation's terms)
            ma0 = np.abs(m["a0"])
            ma1 = (ma0 @ np.abs(p["W1"]).T + np.abs(p["b1"])) * (m["pre1"] > 0)
            ma2 = (ma1 @ np.abs(p["W2"]).T + np.abs(p["b2"])) * (m["pre2"] > 0)
            m2p = (mlog @ np.abs(p["W3"])) * (m["pre2"] > 0)
            m1p = (m2p @ np.abs(p["W2"])) * (m["pre1"] > 0)
            mz_in[:, A] += m1p @ np.abs(p["W1"])
            mags.append([m1p.T @ ma0, m1p.sum(axis=0), m2p.T @ ma1, m2p.sum(axis=0), mlog.T @ ma2,
                         mlog.sum(axis=0)])
        mz = mz_in
    flat = np.concatenate([np.concatenate([t.ravel() for t in gl]) for gl in reversed(grads)])
    if magnitudes:
        mflat = np.concatenate([np.concatenate([t.ravel() for t in gl]) for gl in reversed(mags)])
        return L, flat, logq, mflat
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

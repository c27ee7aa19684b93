"""Helpers of the flow parity tests: random weights, BF16 rounding of the
weights, and the oracle-side distance of every sample to its nearest bin
decision."""
import numpy as np

from oracle import flow as of
from synth import he_init_segments

L, K, H = 4, 32, 64


def bf16(a):
    """Round FP32 values to BF16 (round to nearest even), as FP32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def weights_bf16(theta, dim):
    """Round the W segments (not the biases) to BF16, as the kernels do."""
    th = np.array(theta, dtype=np.float32, copy=True)
    off = 0
    for sh in of.layer_shapes(dim, L, K, H):
        sz = sh["sizes"]
        for k, size in enumerate(sz):
            if k in (0, 2, 4):
                th[off:off + size] = bf16(th[off:off + size])
            off += size
    return th.astype(np.float64)


def random_theta(dim, seed, out_scale=0.1):
    """He-initialised hidden layers, non-zero hidden biases, and output
    weights of standard deviation out_scale: logits of O(1) spread, as in a
    flow part-way through training."""
    rng = np.random.default_rng(seed)
    th = he_init_segments(of.init_segments(dim, L, K, H), seed)
    off = 0
    for sh in of.layer_shapes(dim, L, K, H):
        sz = sh["sizes"]
        o3 = off + sum(sz[:4])
        th[o3:o3 + sz[4] + sz[5]] = rng.normal(0, out_scale, sz[4] + sz[5]).astype(np.float32)
        th[off + sz[0]:off + sz[0] + sz[1]] = rng.normal(0, 0.1, sz[1]).astype(np.float32)
        off += sum(sz)
    return th


def margins(theta, pts, dim, direction, operand=None):
    """Oracle-side distance of every sample to the nearest decision boundary
    over all layers: |z - k/K| for the density direction's bin choice,
    |v - C_k| over the interior cumulative knots for the sampling
    direction's."""
    layers = of.unpack(theta, dim, L, K, H)
    z = np.array(pts, dtype=np.float64, copy=True)
    n = z.shape[0]
    marg = np.full(n, np.inf)
    seq = layers if direction == "density" else list(reversed(layers))
    rows = np.arange(n)
    for p in seq:
        A, B = p["A"], p["B"]
        Q = of._mlp(p, z[:, A], K, operand or of._same)["Q"]
        cum = np.concatenate([np.zeros((n, len(B), 1)), np.cumsum(Q, axis=2)], axis=2)
        for jb, j in enumerate(B):
            if direction == "density":
                t = K * z[:, j]
                marg = np.minimum(marg, np.abs(t - np.round(t)) / K)
                b = np.minimum(np.floor(t).astype(int), K - 1)
                z[:, j] = cum[rows, jb, b] + (t - b) * Q[rows, jb, b]
            else:
                v = z[:, j]
                marg = np.minimum(marg, np.min(np.abs(cum[:, jb, 1:K] - v[:, None]), axis=1))
                b = np.minimum(np.sum(cum[:, jb, 1:K] <= v[:, None], axis=1), K - 1)
                z[:, j] = (b + (v - cum[rows, jb, b]) / Q[rows, jb, b]) / K
    return marg




GAMMA_F32 = 65 * 2.0 ** -24   # error bound of an FP32 dot product of up to 65 terms (64 + bias)


def bf16_operand(jitter=0.0, rng=None):
    """Operand model of the BF16 kernels for the oracle's `operand` hook:
    the FP64 value rounded to FP32 (the kernels' activations and deltas are
    FP32 accumulations), then to BF16 (round to nearest even).  With jitter
    > 0 each value a, formed from terms whose magnitudes sum to mag, is
    first moved by jitter mag xi, xi uniform in (-1, 1): the kernels
    accumulate in another order than NumPy, so their FP32 value of an
    operand differs by up to GAMMA_F32 mag, and one that lies that close to
    a BF16 rounding midpoint can round the other way.  A hidden unit that
    is zero (inactive) stays zero and an active one stays non-negative."""
    def op(a, mag):
        a = np.asarray(a, dtype=np.float64)
        if jitter:
            b = a + jitter * np.asarray(mag) * rng.uniform(-1.0, 1.0, a.shape)
            a = np.where(a > 0, np.maximum(b, 0.0), 0.0) if np.all(a >= 0) else b
        return bf16(a.astype(np.float32)).astype(np.float64)
    return op


def bf16_model(fn, members=16, jitter=GAMMA_F32, seed=0):
    """fn(operand) -> tuple of arrays.  Returns the BF16 operand model's
    outputs (no jitter) and, per output, the root-mean-square over `members`
    jittered evaluations of their departure from it: the scale on which
    the kernels' own accumulation order can move the result."""
    base = fn(bf16_operand())
    rng = np.random.default_rng(seed)
    acc = [np.zeros_like(np.asarray(b, dtype=np.float64)) for b in base]
    for _ in range(members):
        out = fn(bf16_operand(jitter, rng))
        for k, (o, b) in enumerate(zip(out, base)):
            acc[k] += (np.asarray(o) - np.asarray(b)) ** 2
    return base, [np.sqrt(a / members) for a in acc]


class TieRecorder:
    """Operand hook of the BF16 model that also records, per sample, whether
    any operand lies within `rel` of its magnitude of a BF16 rounding
    midpoint: where none does, a kernel whose FP32 operands differ from the
    model's by less than that rounds every operand to the same BF16 value,
    and the two computations differ only by FP32 rounding."""

    def __init__(self, rel=GAMMA_F32):
        self.rel = rel
        self.tie = None

    def __call__(self, a, mag):
        a = np.asarray(a, dtype=np.float64)
        f = a.astype(np.float32)
        low = (f.view(np.uint32) & 0xFFFF).astype(np.int64)
        ulps = np.abs(low - 0x8000).astype(np.float64)       # distance to the midpoint in FP32 ulps
        sp = np.spacing(np.abs(f)).astype(np.float64)
        near = (ulps <= self.rel * np.asarray(mag) / sp + 1.0) & (f != 0)
        t = near.reshape(a.shape[0], -1).any(axis=1)
        self.tie = t if self.tie is None else (self.tie | t)
        return bf16(f).astype(np.float64)

"""Philox-4xW-R counter-based generator (oracle side) — test infrastructure.

Published method: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11.  The thesis leaves the generator unspecified.  One
round on a counter (c0, c1, c2, c3) with key (k0, k1):

    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2      (full 2W-bit products)
    counter'   = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)

and between rounds the key is bumped by the Weyl constants (W0, W1) modulo
2^W.  Ten rounds.

Counter layout used for VEGAS sampling (the same on the GPU side):
    c0 = sample index low 32 bits, c1 = sample index high 32 bits,
    c2 = iteration,                c3 = (stream << 8) | block,
    key = (seed low 32 bits, seed high 32 bits),
where block b supplies the uniforms of dimensions 4b .. 4b+3.
Uniform: u = (k + 1/2) * 2^-32, exact in FP64, strictly inside (0, 1).

Pins (tests/test_oracle_philox.py):
  * philox_generic at W=64 reproduces numpy.random.Philox (Philox-4x64-10,
    an independent implementation of the same published round function);
  * philox4x32 (vectorised) equals philox_generic at W=32 word for word;
  * uniformity of the 32-bit outputs (chi^2 over 1000 bins, mean, variance).
The 4x32 constants themselves have no in-container known-answer vector:
beyond the shared round structure their pin is the GPU/oracle bitwise match.
"""
import numpy as np

MULT = {32: (0xD2511F53, 0xCD9E8D57), 64: (0xD2E7470EE14C6C93, 0xCA5A826395121157)}
WEYL = {32: (0x9E3779B9, 0xBB67AE85), 64: (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)}


def philox_generic(counter, key, width=32, rounds=10):
    """Pure-Python Philox-4xW-R on Python integers (any width 32 or 64)."""
    mask = (1 << width) - 1
    c0, c1, c2, c3 = (int(v) & mask for v in counter)
    k0, k1 = (int(v) & mask for v in key)
    m0, m1 = MULT[width]
    w0, w1 = WEYL[width]
    for r in range(rounds):
        if r:
            k0 = (k0 + w0) & mask
            k1 = (k1 + w1) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> width, p0 & mask
        hi1, lo1 = p1 >> width, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _mulhilo32(m, c):
    p = np.uint64(m) * c.astype(np.uint64)
    return (p >> np.uint64(32)).astype(np.uint32), (p & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=10):
    """Vectorised Philox-4x32-R over uint32 arrays (broadcast)."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint32) for v in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    m0, m1 = MULT[32]
    w0, w1 = WEYL[32]
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = np.uint32((int(k0) + w0) & 0xFFFFFFFF)
                k1 = np.uint32((int(k1) + w1) & 0xFFFFFFFF)
            hi0, lo0 = _mulhilo32(m0, c0)
            hi1, lo1 = _mulhilo32(m1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def to_unit(k):
    """u = (k + 1/2) 2^-32 for uint32 words k (exact in FP64)."""
    return (np.asarray(k, dtype=np.float64) + 0.5) * 2.0 ** -32


def sample_words(seed, stream, iteration, idx, dim):
    """Return the (n, dim) uint32 words of samples with indices idx."""
    idx = np.asarray(idx, dtype=np.uint64)
    lo = (idx & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hi = (idx >> np.uint64(32)).astype(np.uint32)
    k0 = seed & 0xFFFFFFFF
    k1 = (seed >> 32) & 0xFFFFFFFF
    n_blocks = (dim + 3) // 4
    cols = []
    for b in range(n_blocks):
        c3 = np.uint32(((stream << 8) | b) & 0xFFFFFFFF)
        w = philox4x32(lo, hi, np.uint32(iteration), c3, k0, k1)
        cols.extend(w)
    return np.stack(cols[:dim], axis=1)


def sample_uniforms(seed, stream, iteration, idx, dim):
    """Return the (n, dim) FP64 uniforms of samples with indices idx."""
    return to_unit(sample_words(seed, stream, iteration, idx, dim))

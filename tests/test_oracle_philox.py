"""Pins of the oracle's Philox generator (no GPU)."""
import numpy as np
import pytest

from oracle.philox import philox_generic, philox4x32, sample_words, sample_uniforms, to_unit


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((0x0123456789ABCDEF, 0xFEDCBA9876543210), (5, 6, 7, 8)),
    ((2**64 - 1, 2**64 - 1), (2**64 - 3, 2**64 - 1, 2**64 - 1, 2**64 - 1)),
    ((0xDEADBEEF, 42), (123456789, 0, 77, 1 << 63)),
])
def test_generic_64_matches_numpy_philox(key, ctr):
    # numpy's Philox is Philox-4x64-10; it pre-increments its 256-bit counter,
    # so raw words 0..3 are philox(counter + 1) and 4..7 philox(counter + 2).
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    raw = [int(v) for v in bg.random_raw(8)]

    def add(c, k):
        v = sum(int(w) << (64 * i) for i, w in enumerate(c)) + k
        v &= (1 << 256) - 1
        return [(v >> (64 * i)) & (2**64 - 1) for i in range(4)]

    assert list(philox_generic(add(ctr, 1), key, 64)) == raw[:4]
    assert list(philox_generic(add(ctr, 2), key, 64)) == raw[4:]


def test_vectorised_4x32_matches_generic():
    rng = np.random.default_rng(7)
    c = rng.integers(0, 2**32, size=(4, 200), dtype=np.uint64).astype(np.uint32)
    k0, k1 = 0x9ABCDEF0, 0x13579BDF
    w = philox4x32(c[0], c[1], c[2], c[3], k0, k1)
    for i in range(200):
        ref = philox_generic([int(c[r][i]) for r in range(4)], (k0, k1), 32)
        assert tuple(int(w[r][i]) for r in range(4)) == ref


def test_rounds_matter():
    a = philox_generic((1, 2, 3, 4), (5, 6), 32, rounds=10)
    b = philox_generic((1, 2, 3, 4), (5, 6), 32, rounds=7)
    assert a != b


def test_counter_layout_blocks():
    # dims 4..7 come from block 1, i.e. c3 = (stream << 8) | 1
    idx = np.array([0, 1, 2**32 + 5], dtype=np.uint64)
    w = sample_words(seed=0x1122334455667788, stream=3, iteration=9, idx=idx, dim=6)
    for r, i in enumerate(idx):
        i = int(i)
        blk0 = philox_generic((i & 0xFFFFFFFF, i >> 32, 9, (3 << 8) | 0), (0x55667788, 0x11223344), 32)
        blk1 = philox_generic((i & 0xFFFFFFFF, i >> 32, 9, (3 << 8) | 1), (0x55667788, 0x11223344), 32)
        assert [int(v) for v in w[r]] == list(blk0) + list(blk1[:2])


def test_unit_interval_open_and_exact():
    k = np.array([0, 1, 2**31, 2**32 - 1], dtype=np.uint32)
    u = to_unit(k)
    assert u[0] == 2.0**-33 and u[-1] == 1.0 - 2.0**-33
    assert np.all((u > 0) & (u < 1))


def test_uniformity():
    n = 2_000_000
    u = sample_uniforms(seed=0, stream=0, iteration=0, idx=np.arange(n, dtype=np.uint64), dim=4)
    for j in range(4):
        col = u[:, j]
        assert abs(col.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
        assert abs(col.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
        counts = np.bincount(np.minimum((col * 1000).astype(int), 999), minlength=1000)
        chi2 = np.sum((counts - n / 1000) ** 2 / (n / 1000))
        # chi^2 with 999 dof: mean 999, sd ~ 44.7
        assert abs(chi2 - 999) < 5 * 44.7
    # different dimensions are uncorrelated
    c = np.corrcoef(u[:, 0], u[:, 1])[0, 1]
    assert abs(c) < 5 / np.sqrt(n)

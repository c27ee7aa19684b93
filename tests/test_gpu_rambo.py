"""GPU RAMBO and unweighting vs the FP64 oracle (through the C ABI).

Both sides draw the same Philox uniforms, so momenta and weights are
compared event by event.  Bar: |k_gpu - k_oracle| <= 1e-9 sqrt_s and
relative 1e-9 on the weights.  The boost x H_b cancels when the q's are
nearly collinear (the printed transformation, not the kernel), multiplying
the one-ulp differences of log/sin/cos by up to gamma^2 (observed on the
oracle alone: 4e-11 relative in two-body weights over 2e5 events).  Unweighted
index lists are integers: bit-exact.
"""
import math

import numpy as np
import pytest

from oracle import rambo as orb

pytestmark = pytest.mark.gpu

CASES = [
    ([0.0, 0.0], 500.0),
    ([0.0] * 3, 91.2),
    ([0.0] * 4, 1000.0),
    ([0.0] * 10, 2000.0),
    ([173.0, 173.0], 800.0),
    ([80.4, 91.2, 4.7], 300.0),
    ([173.0, 173.0, 0.0, 0.0, 4.7], 1500.0),
    ([1.0] * 9, 30.0),
    ([4.9, 5.0], 10.0),  # near threshold: xi small, Newton from far above the root
    ([30.0, 30.0, 30.0, 9.9], 100.0),
]


def run_gpu(vgx, masses, rs, seed, sid, it, first, n):
    import torch
    mom = torch.empty((4, len(masses), n), dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    vgx.rambo_generate(masses, rs, seed, sid, it, first, mom, w)
    torch.cuda.synchronize()
    return mom.cpu().numpy().transpose(2, 1, 0), w.cpu().numpy()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_rambo_matches_oracle(vgx, case):
    masses, rs = CASES[case]
    n = 20_011  # several blocks and a ragged tail
    print(f"rambo n_part={len(masses)} sqrt_s={rs} masses={masses}", flush=True)
    k, w = run_gpu(vgx, masses, rs, 77, 5, 2, 1_000_003, n)
    kr, wr = orb.generate(77, 5, 2, 1_000_003, n, masses, rs)
    assert np.max(np.abs(k - kr)) <= 1e-9 * rs
    assert np.allclose(w, wr, rtol=1e-9, atol=0)
    # physics checks on the GPU output itself (same conditioning bar)
    assert np.allclose(k.sum(axis=1)[:, 0], rs, rtol=1e-9, atol=0)
    assert np.max(np.abs(k.sum(axis=1)[:, 1:])) <= 1e-9 * rs
    m2 = k[:, :, 0] ** 2 - (k[:, :, 1:] ** 2).sum(axis=2)
    assert np.allclose(m2, np.asarray(masses)[None, :] ** 2, rtol=0, atol=1e-9 * rs * rs)


def test_rambo_edges(vgx):
    import torch
    mom = torch.empty((4, 2, 0), dtype=torch.float64, device="cuda")
    w = torch.empty(0, dtype=torch.float64, device="cuda")
    vgx.rambo_generate([0.0, 0.0], 10.0, 1, 0, 0, 0, mom, w)  # no-op
    one = torch.empty((4, 2, 1), dtype=torch.float64, device="cuda")
    w1 = torch.empty(1, dtype=torch.float64, device="cuda")
    for masses, rs in (([0.0], 10.0), ([0.0] * 11, 10.0), ([6.0, 5.0], 10.0), ([-1.0, 0.0], 10.0),
                       ([0.0, 0.0], 0.0), ([0.0, 0.0], float("nan"))):
        with pytest.raises(vgx.VgxError):
            vgx.rambo_generate(masses, rs, 1, 0, 0, 0, torch.empty((4, len(masses), 1), dtype=torch.float64,
                                                                   device="cuda"), w1)
    vgx.rambo_generate([4.9, 5.0], 10.0, 1, 0, 0, 0, one, w1)  # just above threshold
    k = one.cpu().numpy()[:, :, 0]
    assert np.isclose(k[0].sum(), 10.0, rtol=1e-13)


@pytest.mark.parametrize("n", [1, 4095, 4096, 4097, 300_007])
def test_unweight_bit_exact(vgx, n):
    import torch
    print(f"unweight n={n}", flush=True)
    rng = np.random.default_rng(n)
    w = rng.exponential(1.0, n) * (rng.uniform(size=n) < 0.9)  # with exact zeros
    if n > 10:
        w[3] = -2.0
        w[7] = np.nan
    wt = torch.from_numpy(w).cuda()
    idx = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    k, wm = vgx.unweight(wt, 9, 3, 1, idx)
    ref, wref = orb.unweight(w, 9, 3, 1)
    assert wm == wref
    assert k == ref.size
    assert np.array_equal(idx[:k].cpu().numpy(), ref)
    # a given bound
    k2, wm2 = vgx.unweight(wt, 9, 3, 1, idx, w_max=3.0 * wref)
    ref2, _ = orb.unweight(w, 9, 3, 1, w_max=3.0 * wref)
    assert wm2 == 3.0 * wref and k2 == ref2.size
    assert np.array_equal(idx[:k2].cpu().numpy(), ref2)


@pytest.mark.parametrize("off,n", [(1, 100_000), (1, 100_001), (1, 1), (1, 2), (0, 2), (2, 3)])
def test_unweight_on_offset_views(vgx, off, n):
    """Weights starting off an aligned 16-byte boundary (a view at an odd
    offset), odd and even lengths: the maximum and the kept indices as the
    oracle's."""
    import torch
    print(f"unweight view off={off} n={n}", flush=True)
    w = np.random.default_rng(n + off).exponential(1.0, off + n)
    w[off + n // 2] = 50.0 if n > 2 else w[off + n // 2]  # a maximum inside
    w[-1] = 60.0  # and one at the end: the last weight
    wt = torch.from_numpy(w).cuda()[off:]
    idx = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    k, wm = vgx.unweight(wt, 5, 1, 0, idx)
    ref, wref = orb.unweight(w[off:], 5, 1, 0)
    assert wm == wref == 60.0
    assert k == ref.size and np.array_equal(idx[:k].cpu().numpy(), ref)
    if n > 1:  # and the first weight as the maximum
        w2 = w.copy()
        w2[off] = 70.0
        k, wm = vgx.unweight(torch.from_numpy(w2).cuda()[off:], 5, 1, 0, idx)
        ref, wref = orb.unweight(w2[off:], 5, 1, 0)
        assert wm == wref == 70.0 and k == ref.size
        assert np.array_equal(idx[:k].cpu().numpy(), ref)


def test_unweight_edges(vgx):
    import torch
    idx = torch.empty(10, dtype=torch.int64, device="cuda")
    assert vgx.unweight(torch.zeros(10, dtype=torch.float64, device="cuda"), 1, 0, 0, idx) == (0, 0.0)
    assert vgx.unweight(torch.empty(0, dtype=torch.float64, device="cuda"), 1, 0, 0,
                        torch.empty(0, dtype=torch.int64, device="cuda"))[0] == 0
    k, wm = vgx.unweight(torch.full((10,), 2.0, dtype=torch.float64, device="cuda"), 1, 0, 0, idx)
    assert (k, wm) == (10, 2.0) and np.array_equal(idx.cpu().numpy(), np.arange(10))
    with pytest.raises(vgx.VgxError):
        vgx.unweight(torch.ones(10, dtype=torch.float64, device="cuda"), 1, 0, 0, idx, w_max=-1.0)


def test_rambo_then_unweight_full_size_sampled(vgx):
    """The benchmark launch (1e7 four-particle massive events) checked on a
    sample of events the oracle recomputes, then unweighted on the device and
    compared index for index with the oracle's unweighting of the GPU weights."""
    import torch
    n = 10_000_000
    masses, rs = [173.0, 173.0, 4.7, 0.0], 1500.0
    print(f"rambo full size n={n}", flush=True)
    mom = torch.empty((4, 4, n), dtype=torch.float64, device="cuda")
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    vgx.rambo_generate(masses, rs, 21, 1, 0, 0, mom, w)
    pick = np.sort(np.random.default_rng(4).choice(n, 2000, replace=False))
    kp = mom[:, :, torch.from_numpy(pick).cuda()].cpu().numpy().transpose(2, 1, 0)
    wp = w[torch.from_numpy(pick).cuda()].cpu().numpy()
    for j, e in enumerate(pick[:200]):
        kr, wr = orb.generate(21, 1, 0, int(e), 1, masses, rs)
        assert np.max(np.abs(kp[j] - kr[0])) <= 1e-9 * rs
        assert wp[j] == pytest.approx(wr[0], rel=1e-9)
    idx = torch.empty(n, dtype=torch.int64, device="cuda")
    k, wm = vgx.unweight(w, 21, 2, 0, idx)
    wh = w.cpu().numpy()
    ref, wref = orb.unweight(wh, 21, 2, 0)
    assert wm == wref and k == ref.size
    assert np.array_equal(idx[:k].cpu().numpy(), ref)
    eff = k / n
    assert abs(eff - wh.mean() / wm) < 4 * math.sqrt(eff * (1 - eff) / n)

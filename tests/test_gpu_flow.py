"""GPU coupling flow (MFMA, BF16 operands, FP32 accumulation) vs the oracle.

The oracle evaluates the same network in FP64 with the kernel's BF16 weights
(biases stay FP32 on both sides); the remaining difference is the BF16
rounding of the activations that feed each matrix product (relative 2^-9).
Error model (BF16 mode): each rounded activation carries a relative error
<= 2^-9; through K = 64 terms a logit moves by ~sqrt(64) 2^-9 |W||h| ~ 1e-3,
and log q sums ln(32 Q_b) over 2 L |B| / 2 transforms, a random walk of such
errors.  Bars: median |d log q| <= 5e-3 and 99th percentile <= 3e-2, |d y|
99th percentile <= 2e-3; the loss to 1e-2 relative; gradients to 5e-2 in
relative L2 norm per weight tensor (BF16 deltas too) with overall cosine
similarity > 0.995.  A bin decision flips where a sample lies within the
activation error of a bin edge (density direction) or of a cumulative knot
(sampling direction); there log q jumps, so the percentile bars are taken
over samples whose oracle-side margin exceeds 2e-3, and >= 90% of all
samples must meet |d log q| <= 2e-2 and |d y| <= 2e-3.  Output-layer
weights are drawn with a scale that gives logits of O(1) spread, as in a
flow part-way through training; much larger logits make log q so steep
that the comparison (and g/q itself) is dominated by bin-edge effects.
"""
import math

import numpy as np
import pytest

from oracle import flow as of
from oracle.integrands import gauss, gauss_integral
from oracle.philox import sample_uniforms
from synth import he_init_segments

pytestmark = pytest.mark.gpu

L, K, H = 4, 32, 64


def bf16(a):
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
    rng = np.random.default_rng(seed)
    th = he_init_segments(of.init_segments(dim, L, K, H), seed)
    off = 0
    for sh in of.layer_shapes(dim, L, K, H):
        sz = sh["sizes"]
        o3 = off + sum(sz[:4])
        th[o3:o3 + sz[4] + sz[5]] = rng.normal(0, out_scale, sz[4] + sz[5]).astype(np.float32)
        # non-zero hidden biases exercise the bias path
        th[off + sz[0]:off + sz[0] + sz[1]] = rng.normal(0, 0.1, sz[1]).astype(np.float32)
        off += sum(sz)
    return th


def margins(theta, pts, dim, direction):
    """Oracle-side distance of every sample to the nearest decision boundary
    over all layers (bin edges in z for the density direction, cumulative
    knots for the sampling direction)."""
    layers = of.unpack(theta, dim, L, K, H)
    z = np.array(pts, dtype=np.float64, copy=True)
    n = z.shape[0]
    marg = np.full(n, np.inf)
    seq = layers if direction == "density" else list(reversed(layers))
    for p in seq:
        A, B = p["A"], p["B"]
        Q = of._mlp(p, z[:, A], K)["Q"]
        cum = np.concatenate([np.zeros((n, len(B), 1)), np.cumsum(Q, axis=2)], axis=2)
        for jb, j in enumerate(B):
            if direction == "density":
                t = K * z[:, j]
                marg = np.minimum(marg, np.abs(t - np.round(t)) / K)
                b = np.minimum(np.floor(t).astype(int), K - 1)
                z[:, j] = cum[np.arange(n), jb, b] + (t - b) * Q[np.arange(n), jb, b]
            else:
                v = z[:, j]
                marg = np.minimum(marg, np.min(np.abs(cum[:, jb, 1:K] - v[:, None]), axis=1))
                b = np.minimum(np.sum(cum[:, jb, 1:K] <= v[:, None], axis=1), K - 1)
                z[:, j] = (b + (v - cum[np.arange(n), jb, b]) / Q[np.arange(n), jb, b]) / K
    return marg


def check_bars(dl, dy, safe):
    print(f"  |dlogq| median {np.median(dl[safe]):.2e} p99 {np.percentile(dl[safe], 99):.2e} "
          f"max {dl[safe].max():.2e}; |dy| p99 {np.percentile(dy[safe], 99):.2e}; safe frac {safe.mean():.2f}")
    assert safe.mean() > 0.05  # d = 8: 16 bin decisions per sample
    assert np.median(dl[safe]) <= 5e-3
    assert np.percentile(dl[safe], 99) <= 3e-2
    assert np.percentile(dy[safe], 99) <= 2e-3
    assert np.mean((dl <= 2e-2) & (dy <= 2e-3)) >= 0.9


def make_flow(vgx, dim, theta):
    return vgx.flow_create(dim, theta, L, K, H)


@pytest.mark.parametrize("dim,count", [(3, 29760), (8, 51200), (2, None), (12, None)])
def test_parameter_count_matches_oracle(vgx, dim, count):
    n = vgx.flow_num_params(dim, L, K, H)
    assert n == of.n_params(dim, L, K, H)
    if count:
        assert n == count


@pytest.mark.parametrize("dim", [3, 8])
def test_identity_initialisation(vgx, dim):
    import torch
    print(f"flow identity dim={dim}", flush=True)
    th = he_init_segments(of.init_segments(dim, L, K, H), 0)
    f = make_flow(vgx, dim, th)
    try:
        n = 4099
        y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, n, 5, 1, 0, y, lq)
        torch.cuda.synchronize()
        u = sample_uniforms(5, 1 | (1 << 23), 0, np.arange(n, dtype=np.uint64), dim)
        assert np.max(np.abs(y.cpu().numpy().T - u)) < 2e-7
        assert np.all(lq.cpu().numpy() == 0.0)
    finally:
        vgx.flow_destroy(f)


@pytest.mark.parametrize("dim", [3, 8])
def test_sampling_direction_matches_oracle(vgx, dim):
    import torch
    print(f"flow sample parity dim={dim}", flush=True)
    th = random_theta(dim, 10 + dim)
    thb = weights_bf16(th, dim)
    f = make_flow(vgx, dim, th)
    try:
        n = 20000 + 17
        y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, n, 7, 3, 2, y, lq)
        u = sample_uniforms(7, 3 | (1 << 23), 2, np.arange(n, dtype=np.uint64), dim)
        yr, lqr = of.sample(thb, u, dim, L, K, H)
        dy = np.max(np.abs(y.cpu().numpy().T - yr), axis=1)
        dl = np.abs(lq.cpu().numpy() - lqr)
        m = margins(thb, u, dim, "sampling")
        check_bars(dl, dy, m > 2e-3)
    finally:
        vgx.flow_destroy(f)


@pytest.mark.parametrize("dim", [3, 8])
def test_density_direction_matches_oracle_and_inverts_sampling(vgx, dim):
    import torch
    print(f"flow density parity dim={dim}", flush=True)
    th = random_theta(dim, 20 + dim)
    thb = weights_bf16(th, dim)
    f = make_flow(vgx, dim, th)
    try:
        n = 20000
        rng = np.random.default_rng(dim)
        yy = rng.uniform(size=(n, dim))
        yt = torch.tensor(yy.T.copy(), device="cuda")
        u = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_density(f, yt, lq, u=u)
        ur, lqr = of.density(thb, yy, dim, L, K, H)
        du = np.max(np.abs(u.cpu().numpy().T - ur), axis=1)
        dl = np.abs(lq.cpu().numpy() - lqr)
        check_bars(dl, du, margins(thb, yy, dim, "density") > 2e-3)
        # GPU self-consistency: density(sample(u)) returns u and the same log q
        y2 = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq2 = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, n, 1, 0, 0, y2, lq2)
        u2 = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq3 = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_density(f, y2, lq3, u=u2)
        uref = sample_uniforms(1, 1 << 23, 0, np.arange(n, dtype=np.uint64), dim)
        back = np.max(np.abs(u2.cpu().numpy().T - uref), axis=1)
        same = np.abs(lq3.cpu().numpy() - lq2.cpu().numpy())
        assert np.mean((back < 1e-4) & (same < 1e-4)) > 0.99
    finally:
        vgx.flow_destroy(f)


@pytest.mark.parametrize("dim", [3, 8])
def test_loss_and_gradient_match_oracle(vgx, dim):
    import torch
    print(f"flow gradient parity dim={dim}", flush=True)
    th = random_theta(dim, 30 + dim, out_scale=0.05)
    thb = weights_bf16(th, dim)
    f = make_flow(vgx, dim, th)
    try:
        n = 8192 + 5
        rng = np.random.default_rng(100 + dim)
        yy = rng.uniform(size=(n, dim))
        g = gauss(yy, 0.5, 0.25) + 0.05
        P = vgx.flow_num_params(dim, L, K, H)
        loss, grad = vgx.flow_loss_grad(f, torch.tensor(yy.T.copy(), device="cuda"), torch.tensor(g, device="cuda"), P)
        lr, gr, _ = of.loss_and_grad(thb, yy, g, dim, L, K, H)
        assert loss == pytest.approx(lr, rel=1e-2)
        cos = float(np.dot(grad, gr) / (np.linalg.norm(grad) * np.linalg.norm(gr)))
        assert cos > 0.995
        off = 0
        for sh in of.layer_shapes(dim, L, K, H):
            for k, size in enumerate(sh["sizes"]):
                a, b = grad[off:off + size].astype(np.float64), gr[off:off + size]
                nb = np.linalg.norm(b)
                if nb > 1e-3 * np.linalg.norm(gr):
                    assert np.linalg.norm(a - b) <= 5e-2 * nb, f"segment {k} at {off}"
                off += size
    finally:
        vgx.flow_destroy(f)


def test_adam_matches_oracle(vgx):
    import torch
    dim = 3
    th = random_theta(dim, 1)
    f = make_flow(vgx, dim, th)
    try:
        P = th.size
        rng = np.random.default_rng(0)
        m = np.zeros(P)
        v = np.zeros(P)
        ref = th.astype(np.float64)
        for t in range(1, 4):
            gr = rng.normal(0, 1e-2, P).astype(np.float32)
            vgx.flow_adam(f, torch.tensor(gr, device="cuda"), 1e-3)
            ref, m, v = of.adam_step(ref, m, v, gr.astype(np.float64), t, 1e-3)
        got = vgx.flow_get_params(f, P)
        assert np.allclose(got, ref, rtol=1e-6, atol=1e-7)
    finally:
        vgx.flow_destroy(f)


def test_flow_weights_are_unbiased(vgx):
    """E[f/q] over flow samples equals the integral for any weights: the
    sampler's reported log q is its true density."""
    import torch
    dim = 3
    th = random_theta(dim, 40, out_scale=0.1)
    f = make_flow(vgx, dim, th)
    c, s = 0.45, 0.15
    v = vgx.vegas_create(vgx.GAUSS, dim, 50, 1.5, 0, 0, vgx.F64, np.concatenate([np.full(dim, c), np.full(dim, s)]))
    try:
        n = 2_000_000
        y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, n, 11, 0, 0, y, lq)
        r = vgx.vegas_iterate_points(v, y, lq)
        I = gauss_integral(dim, c, s)
        assert abs(r["mean"] - I) < 4 * math.sqrt(r["var"])
    finally:
        vgx.vegas_destroy(v)
        vgx.flow_destroy(f)


def test_training_reduces_variance(vgx):
    import torch
    dim = 3
    print("flow training 60 steps", flush=True)
    th = he_init_segments(of.init_segments(dim, L, K, H), 2)
    f = make_flow(vgx, dim, th)
    c, s = 0.3, 0.1
    prm = np.concatenate([np.full(dim, c), np.full(dim, s)])
    v = vgx.vegas_create(vgx.GAUSS, dim, 50, 1.5, 3, 0, vgx.F64, prm)
    try:
        n = 16384
        yb = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        gb = torch.empty(n, dtype=torch.float64, device="cuda")
        losses = []
        for step in range(60):
            vgx.vegas_sample(v, 0, n, step, u=yb, g=gb)   # uniform grid: g = f
            losses.append(vgx.flow_train_step(f, yb, gb, 5e-3))
        assert np.mean(losses[-5:]) < 0.5 * np.mean(losses[:3])
        m = 400_000
        y = torch.empty((dim, m), dtype=torch.float64, device="cuda")
        lq = torch.empty(m, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, m, 4, 0, 0, y, lq)
        rf = vgx.vegas_iterate_points(v, y, lq)
        yu = torch.rand((dim, m), dtype=torch.float64, device="cuda")
        ru = vgx.vegas_iterate_points(v, yu, None)
        I = gauss_integral(dim, c, s)
        assert abs(rf["mean"] - I) < 4 * math.sqrt(rf["var"])
        assert rf["var"] < 0.3 * ru["var"]
    finally:
        vgx.vegas_destroy(v)
        vgx.flow_destroy(f)


def test_bad_arguments(vgx):
    with pytest.raises(vgx.VgxError):
        vgx.flow_create(3, np.zeros(10, dtype=np.float32))
    with pytest.raises(vgx.VgxError):
        vgx.flow_create(1, np.zeros(10, dtype=np.float32))
    assert vgx.flow_num_params(13, L, K, H) == -1


def test_full_batch_gradient_matches_oracle(vgx):
    """The training launch at its full size (1e5 samples, d = 8)."""
    import torch
    dim = 8
    print("flow gradient parity full batch 1e5 d=8", flush=True)
    th = random_theta(dim, 77, out_scale=0.05)
    thb = weights_bf16(th, dim)
    f = make_flow(vgx, dim, th)
    try:
        n = 100_000
        rng = np.random.default_rng(5)
        yy = rng.uniform(size=(n, dim))
        g = gauss(yy, 0.5, 0.3) + 0.05
        P = vgx.flow_num_params(dim, L, K, H)
        loss, grad = vgx.flow_loss_grad(f, torch.tensor(yy.T.copy(), device="cuda"), torch.tensor(g, device="cuda"), P)
        lr, gr, _ = of.loss_and_grad(thb, yy, g, dim, L, K, H)
        assert loss == pytest.approx(lr, rel=1e-2)
        cos = float(np.dot(grad, gr) / (np.linalg.norm(grad) * np.linalg.norm(gr)))
        assert cos > 0.995
    finally:
        vgx.flow_destroy(f)


def test_training_is_bit_reproducible(vgx):
    """Every reduction of a training step has a fixed order (tiles within a
    workgroup in wave order, workgroup partials in a fixed tree), so two
    identical trainings end with identical parameters, bit for bit."""
    import torch
    from synth import he_init_segments
    from synth.batch import GAUSS
    print("flow training bit-reproducible", flush=True)
    dim, n = 3, 50_000
    segs = vgx.flow_param_layout(dim)
    n_par = sum(s[2] for s in segs)
    prm = np.concatenate([np.full(dim, 0.4), np.full(dim, 0.12)])
    finals = []
    for _ in range(2):
        v = vgx.vegas_create(GAUSS, dim, 50, 1.5, 3, 0, vgx.F64, prm)
        f = vgx.flow_create(dim, he_init_segments(segs, seed=9))
        try:
            u = torch.empty((dim, n), dtype=torch.float64, device="cuda")
            g = torch.empty(n, dtype=torch.float64, device="cuda")
            losses = []
            for s in range(8):
                vgx.vegas_sample(v, 0, n, 100 + s, u=u, g=g)
                losses.append(vgx.flow_train_step(f, u, g, 1e-3))
            finals.append((losses, vgx.flow_get_params(f, n_par)))
        finally:
            vgx.flow_destroy(f)
            vgx.vegas_destroy(v)
    assert finals[0][0] == finals[1][0]
    assert np.array_equal(finals[0][1], finals[1][1])


def histogram_flow_params(dim, centre, width, sign=-1.0):
    """Parameters of a flow whose networks ignore their inputs (all weight
    matrices zero): layers 0 and 1, which between them transform every
    dimension once, put bin logits sign ((k + 1/2)/K - centre)^2/(2 width^2)
    on their B dims; the other layers are the identity.  q is then a product
    of one-dimensional histograms: a Gaussian shape (sign -1) or its
    opposite, smallest at the centre (sign +1)."""
    th = np.zeros(of.n_params(dim, L, K, H), dtype=np.float32)
    t = (np.arange(K) + 0.5) / K
    logits = (sign * (t - centre) ** 2 / (2 * width ** 2)).astype(np.float32)
    off = 0
    for li, sh in enumerate(of.layer_shapes(dim, L, K, H)):
        sz = sh["sizes"]
        if li < 2:
            o3 = off + sum(sz[:5])
            th[o3:o3 + sz[5]] = np.tile(logits, len(sh["B"]))
        off += sum(sz)
    return th


def test_proposal_worse_than_vegas_signals_fallback(vgx):
    """Plain VEGAS judges a proposal: points from a flow whose variance per
    sample exceeds that of the context's latest plain iteration return
    VGX_EFALLBACK (the unbiased estimate is still recorded); a better flow
    does not.  Target: a d = 3 Gaussian (centre 0.5, width 0.1) on the
    uniform grid, relative variance per sample about 21 for plain VEGAS;
    a flow peaked on the Gaussian (about 0.025) and one shaped the opposite
    way, least dense at the peak (about 108; q is bounded below everywhere,
    so the sample variance is a sound estimate)."""
    import torch
    print("flow: fallback judged by plain VEGAS", flush=True)
    dim, n = 3, 200_000
    c, s = 0.5, 0.1
    v = vgx.vegas_create(vgx.GAUSS, dim, 50, 1.5, 8, 0, vgx.F64,
                         np.concatenate([np.full(dim, c), np.full(dim, s)]))
    good = make_flow(vgx, dim, histogram_flow_params(dim, 0.5, 0.1))
    bad = make_flow(vgx, dim, histogram_flow_params(dim, 0.5, 0.3, sign=1.0))
    try:
        plain = vgx.vegas_iterate(v, n, 0)
        y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(good, n, 9, 0, 0, y, lq)
        rg = vgx.vegas_iterate_points(v, y, lq)
        assert not rg["fallback"]
        vgx.flow_sample(bad, n, 9, 0, 1, y, lq)
        with pytest.raises(vgx.VgxError) as ei:
            vgx.vegas_iterate_points(v, y, lq)
        assert ei.value.status == vgx.VGX_EFALLBACK
        vgx.flow_sample(bad, n, 9, 0, 2, y, lq)
        rb = vgx.vegas_iterate_points(v, y, lq, allow_fallback=True)
        assert rb["fallback"]
        res = vgx.vegas_result(v)
    finally:
        vgx.flow_destroy(good)
        vgx.flow_destroy(bad)
        vgx.vegas_destroy(v)
    rv = lambda r: r["var"] * r["n"] / r["mean"] ** 2
    print(f"  rel. variance per sample: VEGAS {rv(plain):.3g}, good flow {rv(rg):.3g}, bad flow {rv(rb):.3g}")
    assert rv(rg) < rv(plain) < rv(rb)
    I = gauss_integral(dim, c, s)
    assert abs(rg["mean"] - I) < 5 * math.sqrt(rg["var"])
    assert res["n_used"] == 4          # fallback estimates stay in the combination

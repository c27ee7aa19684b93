"""GPU coupling flow (MFMA, BF16 operands, FP32 accumulation) vs the oracle.

Error model (BF16 mode).  The kernels round every matrix-product operand
(layer input, hidden activations, and in training the deltas that meet the
weights) to BF16, 8 significant bits, and accumulate in FP32; the weights
are BF16 on both sides.  The oracle evaluated with that operand rounding
(oracle.flow's `operand` hook with flow_model.bf16_operand: FP64 values
rounded to FP32, then to BF16) is the model of what the kernels compute;
against the plain FP64 oracle it differs by ~1e-3 in ln q per transform
and, where a sample lies within that error of a bin decision, by a whole
bin (sample 11651 of the d = 3 sampling case below: 1.31 in ln q).

The kernels and the model can still round an operand differently where
its FP32 value lies within the accumulation error (at most 65 eps32 of the
sum of its terms' magnitudes) of a BF16 rounding midpoint.  Simulated
under the model (each operand moved by up to that bound before rounding,
8 draws of 20000 samples at d = 3, 8 and 10, before any GPU run), such ties
change ln q by at most 1.5e-2 and y by at most 2.9e-3 on samples farther
than 1e-3 from every decision (the model's own), the gradient by at most
3.7e-3 of a parameter tensor's L2 norm, and leave most samples untouched.
d = 10 (a coupling transforms five coordinates) runs the two-kernel
backward (backward, then weight gradients) instead of the fused one.
Bars, against the model: for every sample farther than 1e-3 from every
decision, |d ln q| <= 5e-2 and |d y| <= 1e-2, and the median sample within
1e-4 (no tie: FP32 agreement); every parameter tensor's gradient (none
skipped) within 1e-2 in relative L2 norm, the loss within 1e-3.  The FP32
operand mode (test_gpu_flow_f32.py) checks the same kernels against the
FP64 oracle at 1e-5 per sample and per gradient element.
"""
import math

import numpy as np
import pytest

from oracle import flow as of
from oracle.integrands import gauss, gauss_integral
from oracle.philox import sample_uniforms
from synth import he_init_segments

from flow_model import H, K, L, bf16_operand, margins, random_theta, weights_bf16

pytestmark = pytest.mark.gpu

MODEL_SAFE = 1e-3   # distance from every decision (model's own) for per-sample bars
BAR_LQ, BAR_Y, BAR_MEDIAN = 5e-2, 1e-2, 1e-4
BAR_SEG, BAR_LOSS = 1e-2, 1e-3


def check_against_model(dl, dy, safe, dl64):
    print(f"  vs BF16 model, samples >= {MODEL_SAFE:.0e} from decisions ({safe.mean():.3f}): |dlogq| max "
          f"{dl[safe].max():.2e} p99 {np.percentile(dl[safe], 99):.2e} median {np.median(dl[safe]):.2e}; |dy| max "
          f"{dy[safe].max():.2e}; vs FP64 (all samples): |dlogq| median {np.median(dl64):.2e} p99 "
          f"{np.percentile(dl64, 99):.2e} max {dl64.max():.2e}", flush=True)
    assert safe.mean() > 0.2
    assert dl[safe].max() <= BAR_LQ
    assert dy[safe].max() <= BAR_Y
    assert np.median(dl[safe]) <= BAR_MEDIAN


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


@pytest.mark.parametrize("dim", [3, 8, 10])
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
        y, lq = y.cpu().numpy().T, lq.cpu().numpy()
    finally:
        vgx.flow_destroy(f)
    u = sample_uniforms(7, 3 | (1 << 23), 2, np.arange(n, dtype=np.uint64), dim)
    ym, lqm = of.sample(thb, u, dim, L, K, H, operand=bf16_operand())
    _, lq64 = of.sample(thb, u, dim, L, K, H)
    safe = margins(thb, u, dim, "sampling", operand=bf16_operand()) > MODEL_SAFE
    check_against_model(np.abs(lq - lqm), np.max(np.abs(y - ym), axis=1), safe, np.abs(lq - lq64))
    if dim == 3:
        # the sample that differs from FP64 by a whole bin: layer 3 puts z_0 in
        # bin 6 (Q = 0.010), whose cumulative knot moves by 1.1e-3 under BF16
        # operands; dividing by K Q moves z_0 by 3.2e-3, across layer 1's knot
        # (2.6e-3 away in FP64): bin 5 (Q = 0.084) for bin 6 (Q = 0.022)
        i = 11651
        assert abs(lqm[i] - lq64[i] - math.log(0.0836 / 0.0224)) < 2e-2
        assert abs(lq[i] - lqm[i]) <= BAR_LQ and abs(lq[i] - lq64[i]) > 1.0


@pytest.mark.parametrize("dim", [3, 8, 10])
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
        um, lqm = of.density(thb, yy, dim, L, K, H, operand=bf16_operand())
        _, lq64 = of.density(thb, yy, dim, L, K, H)
        safe = margins(thb, yy, dim, "density", operand=bf16_operand()) > MODEL_SAFE
        check_against_model(np.abs(lq.cpu().numpy() - lqm), np.max(np.abs(u.cpu().numpy().T - um), axis=1), safe,
                            np.abs(lq.cpu().numpy() - lq64))
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


def check_gradient_against_model(grad, loss, thb, yy, g, dim):
    lm, gm, _ = of.loss_and_grad(thb, yy, g, dim, L, K, H, operand=bf16_operand())
    l64, g64, _ = of.loss_and_grad(thb, yy, g, dim, L, K, H)
    grad = grad.astype(np.float64)
    worst, worst64 = 0.0, 0.0
    off = 0
    for li, sh in enumerate(of.layer_shapes(dim, L, K, H)):
        for k, size in enumerate(sh["sizes"]):
            a, b, c = grad[off:off + size], gm[off:off + size], g64[off:off + size]
            e = np.linalg.norm(a - b) / np.linalg.norm(b)
            worst = max(worst, e)
            worst64 = max(worst64, np.linalg.norm(a - c) / np.linalg.norm(c))
            assert e <= BAR_SEG, f"layer {li} tensor {k}: relative L2 {e:.2e}"
            off += size
    cos64 = float(np.dot(grad, g64) / (np.linalg.norm(grad) * np.linalg.norm(g64)))
    print(f"  vs BF16 model: worst tensor relative L2 {worst:.2e}, loss rel {abs(loss - lm) / lm:.2e}; vs FP64: worst "
          f"tensor {worst64:.2e}, cosine {cos64:.7f}, loss rel {abs(loss - l64) / l64:.2e}", flush=True)
    assert loss == pytest.approx(lm, rel=BAR_LOSS)


@pytest.mark.parametrize("dim", [3, 8, 10])
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
    finally:
        vgx.flow_destroy(f)
    check_gradient_against_model(grad, loss, thb, yy, g, dim)


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
    finally:
        vgx.flow_destroy(f)
    check_gradient_against_model(grad, loss, thb, yy, g, dim)


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


def test_trained_flow_beats_refined_vegas_on_ttbar(vgx, pdf_ctx):
    """What the trained network gains over the method without it, on the
    LO t tbar integrand: the flow, trained on points of a once-refined VEGAS
    grid (weights f J of that grid), has a lower variance per sample than
    plain VEGAS on the same refined grid, and both estimates agree."""
    import torch
    from synth import C2, C4
    print("flow vs refined VEGAS on ttbar", flush=True)
    params = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], 77, 0, vgx.F32, params, pdf=pdf_ctx)
    f = vgx.flow_create(3, he_init_segments(vgx.flow_param_layout(3), C4["seed"]))
    v2 = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], 78, 0, vgx.F32, params, pdf=pdf_ctx)
    try:
        vgx.vegas_iterate(v, 1_000_000, 0)
        vgx.vegas_refine(v)
        n = C4["batch"]
        u = torch.empty((3, n), dtype=torch.float64, device="cuda")
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        losses = []
        for s in range(120):
            vgx.vegas_sample(v, 0, n, 100 + s, u=u, g=g)
            losses.append(vgx.flow_train_step(f, u, g, C4["lr"], sync=(s % 20 == 0 or s == 119)))
        m = 2_000_000
        y = torch.empty((3, m), dtype=torch.float64, device="cuda")
        lq = torch.empty(m, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, m, 5, 0, 0, y, lq)
        rf = vgx.vegas_iterate_points(v, y, lq)
        vgx.vegas_set_grid(v2, vgx.vegas_get_grid(v, 3, C2["n_bins"]))
        rv = vgx.vegas_iterate(v2, m, 0)
    finally:
        vgx.vegas_destroy(v2)
        vgx.flow_destroy(f)
        vgx.vegas_destroy(v)
    rel = lambda r: r["var"] * r["n"] / r["mean"] ** 2
    print(f"  loss {losses[0]:.3f} -> {losses[-1]:.3f}; relative variance per sample: refined VEGAS {rel(rv):.4f},"
          f" trained flow {rel(rf):.4f} ({rel(rv) / rel(rf):.1f}x lower)", flush=True)
    assert losses[-1] < 0.9 * losses[0]
    assert rel(rf) < 0.5 * rel(rv)
    assert abs(rf["mean"] - rv["mean"]) < 4 * math.sqrt(rf["var"] + rv["var"])

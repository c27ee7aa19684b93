"""The flow kernels with FP32 operands (validation mode) against the FP64
oracle: densities, points and every gradient element.

VGX_OPERANDS_F32 runs the same kernels and tile structure as the product
path with FP32 operands (v_mfma_f32_32x32x2_f32), so what remains between
GPU and oracle is FP32 rounding: each network product is a dot product of
at most 65 terms (relative error ~1e-7 for random-signed terms, at most
65 eps32 = 4e-6 of the sum of magnitudes), softmax and ln in FP32 (a few
ulps), the inputs rounded to FP32 (3e-8).  The bars, fixed by the flow
specification of the parity contract and not by these runs: y and ln q
per sample to 1e-5 absolute (y lies in the unit cube; ln q's error is the
relative error of q), the loss to 1e-6 relative, and every gradient
element p to 1e-5 of its magnitude A_p (the gradient formula on absolute
values, oracle.flow.loss_and_grad(magnitudes=True), hidden activations
included: a unit just above zero is a cancellation of its pre-activation's
terms): the scale of the rounding error of any order of evaluation; where
nothing cancels A_p = |g_p| and the bar is 1e-5 relative.

A bin decision can differ where a sample lies within the FP32 error of a
bin edge (density direction) or of a cumulative knot (sampling
direction); samples within 1e-4 of one (100x the error of z) are left out
of the per-sample comparison, and the gradient batches are drawn from
samples at least 1e-4 from every decision (a flipped decision moves a
sample's whole contribution, not a rounding of it).
"""
import numpy as np
import pytest

from oracle import flow as of
from oracle.integrands import gauss
from oracle.philox import sample_uniforms

from flow_model import H, K, L, margins, random_theta

pytestmark = pytest.mark.gpu

SAFE = 1e-4
BAR = 1e-5


def f32_flow(vgx, dim, theta):
    f = vgx.flow_create(dim, theta, L, K, H)
    vgx.flow_set_operands(f, vgx.OPERANDS_F32)
    return f


@pytest.mark.parametrize("dim", [2, 3, 4])
def test_f32_sampling_matches_oracle(vgx, dim):
    import torch
    print(f"flow f32 sampling parity dim={dim}", flush=True)
    th = random_theta(dim, 110 + dim)
    f = f32_flow(vgx, dim, th)
    try:
        n = 20000 + 17
        y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, n, 7, 3, 2, y, lq)
        u = sample_uniforms(7, 3 | (1 << 23), 2, np.arange(n, dtype=np.uint64), dim)
        yr, lqr = of.sample(th.astype(np.float64), u, dim, L, K, H)
        dy = np.max(np.abs(y.cpu().numpy().T - yr), axis=1)
        dl = np.abs(lq.cpu().numpy() - lqr)
        safe = margins(th, u, dim, "sampling") > SAFE
        print(f"  |dlogq| max {dl[safe].max():.2e} p99 {np.percentile(dl[safe], 99):.2e}; |dy| max {dy[safe].max():.2e};"
              f" safe {safe.mean():.4f}; all samples: |dlogq| max {dl.max():.2e}", flush=True)
        assert safe.mean() > 0.9
        assert dl[safe].max() <= BAR
        assert dy[safe].max() <= BAR
    finally:
        vgx.flow_destroy(f)


@pytest.mark.parametrize("dim", [2, 3, 4])
def test_f32_density_matches_oracle(vgx, dim):
    import torch
    print(f"flow f32 density parity dim={dim}", flush=True)
    th = random_theta(dim, 120 + dim)
    f = f32_flow(vgx, dim, th)
    try:
        n = 20000 + 33
        yy = np.random.default_rng(200 + dim).uniform(size=(n, dim))
        u = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_density(f, torch.tensor(yy.T.copy(), device="cuda"), lq, u=u)
        ur, lqr = of.density(th.astype(np.float64), yy, dim, L, K, H)
        du = np.max(np.abs(u.cpu().numpy().T - ur), axis=1)
        dl = np.abs(lq.cpu().numpy() - lqr)
        safe = margins(th, yy, dim, "density") > SAFE
        print(f"  |dlogq| max {dl[safe].max():.2e} p99 {np.percentile(dl[safe], 99):.2e}; |du| max {du[safe].max():.2e};"
              f" safe {safe.mean():.4f}; all samples: |dlogq| max {dl.max():.2e}", flush=True)
        assert safe.mean() > 0.9
        assert dl[safe].max() <= BAR
        assert du[safe].max() <= BAR
    finally:
        vgx.flow_destroy(f)


def safe_batch(th, dim, n, seed):
    """n uniform points of the unit cube at least SAFE from every bin
    decision of the density direction (oracle-side)."""
    rng = np.random.default_rng(seed)
    y = rng.uniform(size=(int(n * 1.25) + 64, dim))
    y = y[margins(th, y, dim, "density") > SAFE]
    assert y.shape[0] >= n
    return np.ascontiguousarray(y[:n])


@pytest.mark.parametrize("dim,n", [(2, 8192 + 5), (3, 8192 + 5), (4, 4096 + 1), (3, 100_000)])
def test_f32_every_gradient_element_matches_oracle(vgx, dim, n):
    import torch
    print(f"flow f32 gradient parity dim={dim} n={n}", flush=True)
    th = random_theta(dim, 130 + dim, out_scale=0.05)
    yy = safe_batch(th, dim, n, 300 + dim)
    g = gauss(yy, 0.5, 0.25) + 0.05
    f = f32_flow(vgx, dim, th)
    try:
        P = vgx.flow_num_params(dim, L, K, H)
        loss, grad = vgx.flow_loss_grad(f, torch.tensor(yy.T.copy(), device="cuda"), torch.tensor(g, device="cuda"), P)
    finally:
        vgx.flow_destroy(f)
    lr, gr, _, mag = of.loss_and_grad(th.astype(np.float64), yy, g, dim, L, K, H, magnitudes=True)
    err = np.abs(grad.astype(np.float64) - gr)
    ratio = np.where(mag > 0, err / np.where(mag > 0, mag, 1.0), np.where(err > 0, np.inf, 0.0))
    clean = (mag > 0) & (np.abs(gr) >= 0.1 * mag)
    rel_clean = err[clean] / np.abs(gr[clean])
    worst = int(np.argmax(ratio))
    print(f"  loss rel {abs(loss - lr) / lr:.2e}; |dg|/A max {ratio.max():.2e} (element {worst}, g {gr[worst]:.3e},"
          f" A {mag[worst]:.3e}) p99 {np.percentile(ratio, 99):.2e}; elements without cancellation"
          f" ({clean.mean():.2f}): relative max {rel_clean.max():.2e}", flush=True)
    assert loss == pytest.approx(lr, rel=1e-6)
    assert np.all(ratio <= BAR)


def test_f32_mode_needs_the_weights_in_lds(vgx):
    """d = 8 with four layers: 4 x 13312 FP32 weights exceed the LDS; the
    call fails and the flow keeps running with BF16 operands."""
    import torch
    from synth import he_init_segments
    dim = 8
    f = vgx.flow_create(dim, he_init_segments(of.init_segments(dim, L, K, H), 3))
    try:
        with pytest.raises(vgx.VgxError) as ei:
            vgx.flow_set_operands(f, vgx.OPERANDS_F32)
        assert ei.value.status == vgx.VGX_EINVAL
        n = 1000
        y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, n, 1, 0, 0, y, lq)
        torch.cuda.synchronize()
        assert np.all(lq.cpu().numpy() == 0.0)  # identity initialisation
    finally:
        vgx.flow_destroy(f)


def test_f32_and_bf16_modes_switch_back(vgx):
    """Switching to FP32 operands and back gives the BF16 results again, bit
    for bit (the packs are rebuilt from the same master weights)."""
    import torch
    dim, n = 3, 5000
    th = random_theta(dim, 141)
    f = vgx.flow_create(dim, th, L, K, H)
    try:
        outs = []
        for mode in (vgx.OPERANDS_BF16, vgx.OPERANDS_F32, vgx.OPERANDS_BF16):
            vgx.flow_set_operands(f, mode)
            y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
            lq = torch.empty(n, dtype=torch.float64, device="cuda")
            vgx.flow_sample(f, n, 2, 0, 0, y, lq)
            outs.append(lq.cpu().numpy())
        assert np.array_equal(outs[0], outs[2])
        assert not np.array_equal(outs[0], outs[1])
    finally:
        vgx.flow_destroy(f)

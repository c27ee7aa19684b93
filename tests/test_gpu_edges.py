"""Edge cases of the GPU path against the oracle or against itself:
bin-count extremes, ragged batches of the hadronic integrands, and ragged
flow batches (tile pairs of 64 samples)."""
import math

import numpy as np
import pytest

from oracle import drellyan, singletop, ttbar, vegas as ov
from oracle.integrands import gauss
from oracle.philox import sample_uniforms
from synth import C2, C5, C6, he_init_segments

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nb", [2, 256])
def test_bin_count_extremes(vgx, nb):
    """An iteration and a refinement with the fewest and the most bins."""
    print(f"edges: n_bins={nb}", flush=True)
    dim, n = 3, 20_003
    prm = np.concatenate([np.full(dim, 0.4), np.full(dim, 0.15)])
    v = vgx.vegas_create(vgx.GAUSS, dim, nb, 1.5, 11, 0, vgx.F64, prm)
    try:
        r = vgx.vegas_iterate(v, n, 0)
        h = vgx.vegas_get_hist(v, dim, nb)
        vgx.vegas_refine(v)
        e_gpu = vgx.vegas_get_grid(v, dim, nb)
    finally:
        vgx.vegas_destroy(v)
    e = ov.uniform_grid(dim, nb)
    u = sample_uniforms(11, 0, 0, np.arange(n, dtype=np.uint64), dim)
    x, jac, idx = ov.vegas_map(u, e)
    w = gauss(x, np.full(dim, 0.4), np.full(dim, 0.15)) * jac
    assert r["s1"] == pytest.approx(math.fsum(w), rel=1e-12)
    assert r["s2"] == pytest.approx(math.fsum(w * w), rel=1e-12)
    for j in range(dim):
        hj = np.bincount(idx[:, j], weights=w * w, minlength=nb)
        assert np.allclose(h[j], hj, rtol=1e-12, atol=1e-300)
    e_ref = ov.refine(e, h, 1.5)
    assert np.allclose(e_gpu, e_ref, rtol=0, atol=1e-12)


def _hadronic(vgx, kind):
    if kind == "ttbar":
        p = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])
        f = lambda x, g: ttbar.integrand(x, g, C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"])
        return vgx.TTBAR, p, f
    if kind == "drellyan":
        p = np.array([C5["sqrt_s"], C5["m_lo"], C5["m_hi"], C5["m_z"], C5["gamma_z"], C5["sw2"], C5["alpha_em"],
                      C5["gev2_to_pb"]])
        return vgx.DRELLYAN, p, lambda x, g: drellyan.integrand_from_config(x, g, C5)
    p = np.array([C6["sqrt_s"], C6["m_top"], C6["m_w"], C6["gamma_w"], C6["sw2"], C6["alpha_em"], C6["gev2_to_pb"]])
    return vgx.SINGLETOP, p, lambda x, g: singletop.integrand_from_config(x, g, C6)


@pytest.mark.parametrize("kind", ["ttbar", "drellyan", "singletop"])
@pytest.mark.parametrize("n", [2, 257, 3001])
def test_hadronic_ragged_iterations(vgx, pdf_ctx, c1_grid, kind, n):
    """Iterations shorter than a workgroup, one past a workgroup, and ragged
    against the grid-stride loop: the sums against the oracle (FP32
    integrand bar)."""
    print(f"edges: {kind} n={n}", flush=True)
    k, p, f = _hadronic(vgx, kind)
    v = vgx.vegas_create(k, 3, 50, 1.5, 21, 3, vgx.F32, p, pdf=pdf_ctx)
    try:
        r = vgx.vegas_iterate(v, n, 2)
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(21, 3, 2, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, ov.uniform_grid(3, 50))
    w = f(x, c1_grid) * jac
    assert r["n"] == n
    assert r["s1"] == pytest.approx(math.fsum(w), rel=1e-5, abs=1e-7 * np.mean(np.abs(w)) * n)
    assert r["s2"] == pytest.approx(math.fsum(w * w), rel=2e-5, abs=1e-7 * np.mean(w * w) * n)


@pytest.mark.parametrize("dim", [3, 8])
def test_flow_ragged_batches_are_prefix_consistent(vgx, dim):
    """Flow samples are counter-based and per-sample: a batch of n points
    equals the first n points of a longer batch, for n below, at and past
    the 64-sample tile pairs, bit for bit; likewise the density direction."""
    import torch
    print(f"edges: flow ragged dim={dim}", flush=True)
    f = vgx.flow_create(dim, he_init_segments(vgx.flow_param_layout(dim), 9))
    try:
        N = 1000
        y = torch.empty((dim, N), dtype=torch.float64, device="cuda")
        lq = torch.empty(N, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, N, 3, 4, 1, y, lq)
        for n in (1, 63, 64, 65, 129):
            ys = torch.empty((dim, n), dtype=torch.float64, device="cuda")
            ls = torch.empty(n, dtype=torch.float64, device="cuda")
            vgx.flow_sample(f, n, 3, 4, 1, ys, ls)
            assert torch.equal(ys, y[:, :n].contiguous())
            assert torch.equal(ls, lq[:n])
        # the density direction on ragged batches: the same per-point values
        ld = torch.empty(N, dtype=torch.float64, device="cuda")
        vgx.flow_density(f, y, ld)
        for n in (1, 63, 65):
            ln = torch.empty(n, dtype=torch.float64, device="cuda")
            vgx.flow_density(f, y[:, :n].contiguous(), ln)
            assert torch.equal(ln, ld[:n])
    finally:
        vgx.flow_destroy(f)


def test_binding_rejects_short_buffers(vgx):
    """Device buffers shorter than the call needs are refused in the binding,
    before any kernel can write or read past them."""
    import torch
    from synth.batch import GAUSS
    from synth import he_init_segments
    v = vgx.vegas_create(GAUSS, 3, 20, 1.5, 1, 0, vgx.F64, np.array([0.5] * 3 + [0.1] * 3))
    try:
        assert vgx.vegas_shape(v) == (3, 20)
        with pytest.raises(ValueError):
            vgx.vegas_sample(v, 0, 100, 0, u=torch.empty((2, 100), dtype=torch.float64, device="cuda"))
        with pytest.raises(ValueError):
            vgx.vegas_iterate_points(v, torch.empty((2, 100), dtype=torch.float64, device="cuda"))
    finally:
        vgx.vegas_destroy(v)
    segs = vgx.flow_param_layout(3)
    f = vgx.flow_create(3, he_init_segments(segs, seed=1))
    try:
        dim, n_par = vgx.flow_shape(f)
        assert dim == 3 and n_par == sum(s[2] for s in segs)
        with pytest.raises(ValueError):
            vgx.flow_sample(f, 100, 1, 0, 0, torch.empty((2, 100), dtype=torch.float64, device="cuda"),
                            torch.empty(100, dtype=torch.float64, device="cuda"))
        with pytest.raises(ValueError):
            vgx.flow_adam(f, torch.zeros(n_par - 1, dtype=torch.float32, device="cuda"), 1e-3)
    finally:
        vgx.flow_destroy(f)


@pytest.mark.parametrize("bad", ["nan", "-inf"])
def test_non_finite_points_iteration_is_reported_and_excluded(vgx, bad):
    """An iteration whose estimate is not finite returns VGX_ENUMERIC and is
    left out of the inverse-variance combination; later finite iterations
    combine as if it had not happened.  The non-finite weight comes from
    caller points with log q = NaN (or -inf: q = 0, an infinite weight)."""
    import torch
    print(f"edges: non-finite points iteration ({bad})", flush=True)
    dim, n, nb = 3, 20_000, 50
    prm = np.concatenate([np.full(dim, 0.45), np.full(dim, 0.2)])
    v = vgx.vegas_create(vgx.GAUSS, dim, nb, 1.5, 5, 0, vgx.F64, prm)
    try:
        r0 = vgx.vegas_iterate(v, n, 0)
        vgx.vegas_refine(v)
        y = torch.rand((dim, n), dtype=torch.float64, device="cuda",
                       generator=torch.Generator(device="cuda").manual_seed(3))
        lq = torch.zeros(n, dtype=torch.float64, device="cuda")
        lq[17] = float(bad)
        with pytest.raises(vgx.VgxError) as ei:
            vgx.vegas_iterate_points(v, y, lq)
        assert ei.value.status == vgx.VGX_ENUMERIC
        mid = vgx.vegas_result(v)
        r2 = vgx.vegas_iterate(v, n, 2)
        res = vgx.vegas_result(v)
        recs = vgx.vegas_results(v)
    finally:
        vgx.vegas_destroy(v)
    assert len(recs) == 3 and not math.isfinite(recs[1]["mean"] + recs[1]["var"])
    # one record: the weighted average (E/var)/(1/var) returns E to rounding
    assert mid["n_used"] == 1 and mid["mean"] == pytest.approx(r0["mean"], rel=1e-15)
    assert res["n_used"] == 2
    m, s, c = ov.combine([r0["mean"], r2["mean"]], [r0["var"], r2["var"]])
    assert res["mean"] == pytest.approx(m, rel=1e-14)
    assert res["sigma"] == pytest.approx(s, rel=1e-14)
    assert res["chi2_dof"] == pytest.approx(c, rel=1e-12, abs=1e-15)


def test_non_finite_integrand_iteration_leaves_the_grid(vgx):
    """An FP32 Gaussian whose normalisation overflows FP32 (sigma = 1e-40 in
    one dimension: the FP32 normalisation and inverse width are infinite,
    infinity times exp(-infinity)) gives NaN weights in a
    plain iteration: VGX_ENUMERIC, nothing combined, and the refinement
    leaves every dimension of the grid unchanged (its histogram is NaN)."""
    print("edges: non-finite plain iteration (FP32 overflow)", flush=True)
    dim, n, nb = 3, 20_000, 50
    prm = np.array([0.5, 0.5, 0.5, 0.2, 1e-40, 0.2])
    v = vgx.vegas_create(vgx.GAUSS, dim, nb, 1.5, 5, 0, vgx.F32, prm)
    try:
        vgx.vegas_set_grid(v, np.tile(np.linspace(0.0, 1.0, nb + 1) ** 1.3, (dim, 1)))
        e0 = vgx.vegas_get_grid(v, dim, nb)
        with pytest.raises(vgx.VgxError) as ei:
            vgx.vegas_iterate(v, n, 0)
        assert ei.value.status == vgx.VGX_ENUMERIC
        assert np.isnan(vgx.vegas_get_hist(v, dim, nb)).all()
        vgx.vegas_refine(v)
        e1 = vgx.vegas_get_grid(v, dim, nb)
        res = vgx.vegas_result(v)
    finally:
        vgx.vegas_destroy(v)
    assert np.array_equal(e1, e0)
    assert res["n_used"] == 0

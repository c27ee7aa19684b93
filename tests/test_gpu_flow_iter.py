"""The fused flow-sampling VEGAS iteration (flow_vegas_iterate) against the
two-step path (flow_sample, then vegas_iterate_points with the points' ln q).

The fused kernel draws the points flow_sample draws (the same Philox
counters and coupling layers) and weights each one by the same operations
on the same values as the iteration kernel does with caller points,
w = f(G(y)) J_G(y) exp(-ln q); only the order of the compensated sums S1 =
sum w and S2 = sum w^2 differs (lanes and workgroups split the samples
differently).  With Neumaier sums over at most ~1e6 weights of one sign
(or a few signs) the two orders agree to a few units of 1e-16 relative; the
bar is 1e-12.  The per-sample pieces are pinned to the FP64 oracle
elsewhere: the flow's points and ln q in test_gpu_flow.py, the weights of
caller points in test_gpu_vegas.py and test_gpu_ttbar.py.
"""
import numpy as np
import pytest

from synth import C2, he_init_segments

pytestmark = pytest.mark.gpu

REL = 1e-12


def _two_step(vgx, f, v, n, seed, sid, it):
    import torch
    dim, _ = vgx.flow_shape(f)
    y = torch.empty((dim, n), dtype=torch.float64, device="cuda")
    lq = torch.empty(n, dtype=torch.float64, device="cuda")
    vgx.flow_sample(f, n, seed, sid, it, y, lq)
    torch.cuda.synchronize()
    return vgx.vegas_iterate_points(v, y, lq, allow_fallback=True)


def _compare(label, fused, ref):
    for k in ("s1", "s2", "mean", "var"):
        a, b = fused[k], ref[k]
        rel = abs(a - b) / max(abs(b), 1e-300)
        print(f"  {label} {k}: fused {a:.17g} two-step {b:.17g} rel {rel:.1e}", flush=True)
        assert rel <= REL, (label, k, a, b)
    assert fused["n"] == ref["n"]


def _flow(vgx, dim, seed):
    return vgx.flow_create(dim, he_init_segments(vgx.flow_param_layout(dim), seed))


@pytest.mark.parametrize("n", [1_000_003, 2, 63, 65, 64 * 4096 + 1])
def test_fused_iteration_matches_two_step_on_ttbar(vgx, c1_grid, n):
    print(f"fused flow iteration ttbar n={n}", flush=True)
    pdf = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    params = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], 77, 0, vgx.F32, params, pdf=pdf)
    f = _flow(vgx, 3, 5)
    try:
        vgx.vegas_iterate(v, 200_000, 0)
        vgx.vegas_refine(v)
        fused = vgx.flow_vegas_iterate(f, v, n, 11, 3, 7, allow_fallback=True)
        ref = _two_step(vgx, f, v, n, 11, 3, 7)
        _compare("ttbar", fused, ref)
    finally:
        vgx.flow_destroy(f)
        vgx.vegas_destroy(v)
        vgx.pdf_destroy(pdf)


@pytest.mark.parametrize("dim,prec", [(2, "F64"), (5, "F32"), (8, "F64")])
def test_fused_iteration_matches_two_step_on_gauss(vgx, dim, prec):
    print(f"fused flow iteration gauss dim={dim} {prec}", flush=True)
    prm = np.concatenate([np.full(dim, 0.5), np.full(dim, 0.2)])
    v = vgx.vegas_create(vgx.GAUSS, dim, 50, 1.5, 3, 0, getattr(vgx, prec), prm)
    f = _flow(vgx, dim, 9)
    try:
        vgx.vegas_iterate(v, 100_000, 0)
        vgx.vegas_refine(v)
        n = 300_017
        fused = vgx.flow_vegas_iterate(f, v, n, 4, 0, 1, allow_fallback=True)
        ref = _two_step(vgx, f, v, n, 4, 0, 1)
        _compare(f"gauss{dim}", fused, ref)
    finally:
        vgx.flow_destroy(f)
        vgx.vegas_destroy(v)


def test_fused_iteration_rejects_what_it_cannot_run(vgx):
    prm = np.concatenate([np.full(3, 0.5), np.full(3, 0.2)])
    v = vgx.vegas_create(vgx.GAUSS, 3, 50, 1.5, 3, 0, vgx.F64, prm)
    f2 = _flow(vgx, 2, 1)
    f3 = _flow(vgx, 3, 1)
    try:
        with pytest.raises(vgx.VgxError) as e:
            vgx.flow_vegas_iterate(f2, v, 1000, 1, 0, 0)
        assert e.value.status == vgx.VGX_EINVAL and "dimension" in str(e.value)
        with pytest.raises(vgx.VgxError) as e:
            vgx.flow_vegas_iterate(f3, v, 1, 1, 0, 0)
        assert e.value.status == vgx.VGX_EINVAL
        vgx.flow_set_operands(f3, vgx.OPERANDS_F32)
        with pytest.raises(vgx.VgxError) as e:
            vgx.flow_vegas_iterate(f3, v, 1000, 1, 0, 0)
        assert e.value.status == vgx.VGX_EINVAL and "BF16" in str(e.value)
        vgx.flow_set_operands(f3, vgx.OPERANDS_BF16)
        r = vgx.flow_vegas_iterate(f3, v, 1000, 1, 0, 0, allow_fallback=True)
        assert r["n"] == 1000 and np.isfinite(r["mean"])
    finally:
        vgx.flow_destroy(f2)
        vgx.flow_destroy(f3)
        vgx.vegas_destroy(v)

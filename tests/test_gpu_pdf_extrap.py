"""GPU behaviour outside the PDF grid and below the alpha_s table (error,
freeze and continuation modes) vs the oracle, through the C ABI.

Bars: FP64 outputs |a - b| <= 1e-10 |b| + 1e-10 max_f |b_f| (the log-branch
continuation multiplies rounding by up to 2|t|, |t| up to a few hundred grid
spacings here).  FP32 outputs are computed in FP64 from the FP32 copy of the
node values; the continuation amplifies that input rounding without bound
where xf(x, Q^2_min) nears zero (gamma = G0'/G0), so they are compared with
the oracle evaluated on the same FP32-rounded node values and rounded to
FP32: 2e-6 of the same scale.  (In-grid FP32 accuracy against the FP64 grid
is covered by test_gpu_pdf.)
"""
import math

import numpy as np
import pytest

from oracle import pdf_extrap as pe
from synth import synthetic_alphas, PdfGridData

pytestmark = pytest.mark.gpu


def queries(grid, rng, n, far):
    x0, x1 = grid.x_knots[0], grid.x_knots[-1]
    q0, q1 = grid.q2_knots[0][0], grid.q2_knots[-1][-1]
    lx_in = rng.uniform(math.log(x0), math.log(x1), n)
    lq_in = rng.uniform(math.log(q0), math.log(q1), n)
    lx_lo = math.log(x0) - rng.uniform(0.0, far, n)
    lq_lo = math.log(q0) - rng.uniform(0.0, far, n)
    lq_hi = math.log(q1) + rng.uniform(0.0, far, n)
    xs = np.exp(np.concatenate([lx_in, lx_lo, lx_in, lx_in, lx_lo, lx_lo]))
    qs = np.exp(np.concatenate([lq_in, lq_in, lq_hi, lq_lo, lq_hi, lq_lo]))
    edge_x = np.array([x0, x0 * (1 - 1e-15), x1, grid.x_knots[1], 1.5, 2.0])
    edge_q = np.array([q0, q0 * (1 - 1e-15), q1, q1 * (1 + 1e-15), grid.q2_knots[1][0], 0.3])
    X, Q = np.meshgrid(edge_x, edge_q)
    bad_x = np.array([0.0, -1e-3, np.nan, 0.5, 0.5, 0.5, np.inf])
    bad_q = np.array([100.0, 100.0, 100.0, 0.0, -5.0, np.inf, 100.0])
    return np.concatenate([xs, X.ravel(), bad_x]), np.concatenate([qs, Q.ravel(), bad_q])


@pytest.mark.parametrize("out", ["f64", "f32"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_extrapolation_matches_oracle(vgx, c1_grid, mode, out):
    import torch
    print(f"pdf extrapolation mode={mode} out={out}", flush=True)
    ctx = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    try:
        vgx.pdf_set_extrapolation(ctx, mode)
        rng = np.random.default_rng(40 + mode)
        tol = 1e-10 if out == "f64" else 2e-6
        x, q2 = queries(c1_grid, rng, 3000, 25.0)
        dt = torch.float64 if out == "f64" else torch.float32
        res = torch.full((11, x.size), 7.0, dtype=dt, device="cuda")
        vgx.pdf_interp(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q2).cuda(), res)
        got = res.double().cpu().numpy()
        if out == "f64":
            ref = pe.interp_extrap(c1_grid, x, q2, mode)
        else:
            g32 = PdfGridData(x_knots=c1_grid.x_knots, q2_knots=c1_grid.q2_knots,
                              xf=[v.astype(np.float32).astype(np.float64) for v in c1_grid.xf],
                              params={}, lambda_qcd=c1_grid.lambda_qcd, q0=c1_grid.q0)
            with np.errstate(over="ignore"):
                ref = pe.interp_extrap(g32, x, q2, mode).astype(np.float32).astype(np.float64)
        nan = np.isnan(ref)
        assert np.array_equal(np.isnan(got), nan)
        assert np.array_equal(nan.all(axis=0), nan.any(axis=0))
        assert vgx.pdf_out_of_range(ctx) == int(nan.all(axis=0).sum())
        fin = ~nan.all(axis=0)
        g, r = got[:, fin], ref[:, fin]
        assert np.array_equal(np.isinf(g), np.isinf(r))
        g, r = np.where(np.isinf(g), 0.0, g), np.where(np.isinf(r), 0.0, r)
        scale = np.abs(r).max(axis=0)[None, :]
        bad = np.abs(g - r) > tol * np.abs(r) + tol * scale
        assert not bad.any(), f"worst {np.abs(g - r)[bad].max():.3e} at {np.argwhere(bad)[:3]}"
        if mode == 0:
            assert nan.all(axis=0).sum() > 5 * 3000
    finally:
        vgx.pdf_destroy(ctx)


def test_mode_switch_and_errors(vgx, c1_grid):
    import torch
    ctx = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    try:
        with pytest.raises(vgx.VgxError):
            vgx.pdf_set_extrapolation(ctx, 3)
        x = torch.tensor([1e-12, 0.5], dtype=torch.float64, device="cuda")
        q2 = torch.tensor([100.0, 1e14], dtype=torch.float64, device="cuda")
        res = torch.empty((11, 2), dtype=torch.float64, device="cuda")
        for mode, finite in ((2, True), (0, False), (1, True)):
            vgx.pdf_set_extrapolation(ctx, mode)
            vgx.pdf_interp(ctx, x, q2, res)
            assert bool(np.isfinite(res.cpu().numpy()).all()) == finite
            assert vgx.pdf_out_of_range(ctx) == (0 if finite else 2)
    finally:
        vgx.pdf_destroy(ctx)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_alphas_extrapolation_matches_oracle(vgx, c1_grid, mode):
    import torch
    print(f"alpha_s extrapolation mode={mode}", flush=True)
    table = synthetic_alphas(c1_grid)
    ctx = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    try:
        vgx.pdf_set_alphas(ctx, table.q2_knots, table.values)
        vgx.pdf_set_extrapolation(ctx, mode)
        lo, hi = table.q2_knots[0][0], table.q2_knots[-1][-1]
        rng = np.random.default_rng(7)
        q2 = np.concatenate([np.exp(rng.uniform(math.log(lo) - 8.0, math.log(hi) + 3.0, 20_000)),
                             [lo, lo * (1 - 1e-15), hi, 0.0, -1.0, np.nan, np.inf]])
        out = torch.empty(q2.size, dtype=torch.float64, device="cuda")
        vgx.pdf_alphas(ctx, torch.from_numpy(q2).cuda(), out)
        got = out.cpu().numpy()
        ref = pe.alphas_extrap(table, q2, mode)
        nan = np.isnan(ref)
        assert np.array_equal(np.isnan(got), nan)
        assert np.allclose(got[~nan], ref[~nan], rtol=1e-13, atol=0)
    finally:
        vgx.pdf_destroy(ctx)

"""Multi-member PDF evaluation (pdf_create_set / pdf_interp_members) vs the
FP64 oracle applied member by member.  Bars as in test_gpu_pdf: FP64 outputs
r_i <= 1e-13, FP32 outputs (from the FP32 node copy) r_i <= 1e-5, with the
stencil-scale floor where the stencil cancels."""
import numpy as np
import pytest

from oracle import pdf as opdf
from synth import C7, PdfGridData, fk_points, pdf_queries, synthetic_pdf_replicas
from test_gpu_pdf import check, stencil_scale

pytestmark = pytest.mark.gpu


def member_grid(base, xf):
    return PdfGridData(x_knots=base.x_knots, q2_knots=base.q2_knots, xf=xf, params={}, lambda_qcd=base.lambda_qcd,
                       q0=base.q0)


@pytest.mark.parametrize("out", ["f64", "f32"])
def test_members_match_oracle(vgx, c1_grid, out):
    import torch
    print(f"pdf members M=7 out={out}", flush=True)
    members = synthetic_pdf_replicas(c1_grid, 7, C7["eps"], C7["seed"])
    ctx = vgx.pdf_create_set(c1_grid.x_knots, c1_grid.q2_knots, members)
    try:
        assert vgx.pdf_shape(ctx) == (11, 7)
        xf_, qf_ = fk_points(C7)
        xr, qr = pdf_queries(3001, seed=99)
        x = np.concatenate([xf_, xr, [1e-12, 0.5]])
        q2 = np.concatenate([qf_, qr, [10.0, 0.3]])  # two points outside the grid
        dt = torch.float64 if out == "f64" else torch.float32
        res = torch.empty((7, 11, x.size), dtype=dt, device="cuda")
        vgx.pdf_interp_members(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q2).cuda(), res)
        got = res.double().cpu().numpy()
        assert vgx.pdf_out_of_range(ctx) == 2
        tol = 1e-13 if out == "f64" else 1e-5
        for m in range(7):
            g = member_grid(c1_grid, members[m])
            ref = opdf.interp(g, x, q2)
            nan = np.isnan(ref)
            assert np.array_equal(np.isnan(got[m]), nan) and nan.any(axis=0).sum() == 2
            ok, r = check(got[m][:, ~nan[0]], ref[:, ~nan[0]], stencil_scale(g, x[~nan[0]], q2[~nan[0]]), tol)
            assert ok.all(), f"member {m}: worst r_i {r[~ok].max():.3e}"
        # member 0 is what pdf_interp evaluates, bit for bit
        one = torch.empty((11, x.size), dtype=dt, device="cuda")
        vgx.pdf_interp(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q2).cuda(), one)
        assert np.array_equal(one.double().cpu().numpy(), got[0], equal_nan=True)
        vgx.pdf_out_of_range(ctx)
    finally:
        vgx.pdf_destroy(ctx)


def test_single_member_set_equals_plain_context(vgx, c1_grid, pdf_ctx):
    import torch
    ctx = vgx.pdf_create_set(c1_grid.x_knots, c1_grid.q2_knots, [c1_grid.xf])
    try:
        x, q2 = pdf_queries(5000, seed=5)
        xt, qt = torch.from_numpy(x).cuda(), torch.from_numpy(q2).cuda()
        a = torch.empty((1, 11, x.size), dtype=torch.float64, device="cuda")
        b = torch.empty((11, x.size), dtype=torch.float64, device="cuda")
        vgx.pdf_interp_members(ctx, xt, qt, a)
        vgx.pdf_interp(pdf_ctx, xt, qt, b)
        assert np.array_equal(a[0].cpu().numpy(), b.cpu().numpy())
        with pytest.raises(ValueError):  # the binding checks the output size
            vgx.pdf_interp(pdf_ctx, xt, qt, torch.empty((10, x.size), dtype=torch.float64, device="cuda"))
        with pytest.raises(ValueError):
            vgx.pdf_interp_members(ctx, xt, qt, torch.empty((11, x.size - 1), dtype=torch.float64, device="cuda"))
    finally:
        vgx.pdf_destroy(ctx)


def test_full_fk_configuration_sampled(vgx, c1_grid):
    """400 members at the 2415 points (the benchmark launch): three members
    checked against the oracle over all points."""
    import torch
    n_rep = max(C7["n_rep"])
    print(f"pdf members full size M={n_rep}", flush=True)
    members = synthetic_pdf_replicas(c1_grid, n_rep, C7["eps"], C7["seed"])
    ctx = vgx.pdf_create_set(c1_grid.x_knots, c1_grid.q2_knots, members)
    try:
        x, q2 = fk_points(C7)
        res = torch.empty((n_rep, 11, x.size), dtype=torch.float64, device="cuda")
        vgx.pdf_interp_members(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(q2).cuda(), res)
        got = res.cpu().numpy()
        assert np.isfinite(got).all() and vgx.pdf_out_of_range(ctx) == 0
        for m in (0, 137, n_rep - 1):
            g = member_grid(c1_grid, members[m])
            ok, r = check(got[m], opdf.interp(g, x, q2), stencil_scale(g, x, q2), 1e-13)
            assert ok.all()
    finally:
        vgx.pdf_destroy(ctx)

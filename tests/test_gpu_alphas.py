"""GPU alpha_s(Q) interpolation (pdf_set_alphas / pdf_alphas) vs the oracle."""
import numpy as np
import pytest

from oracle import alphas as oa
from synth import synthetic_alphas

pytestmark = pytest.mark.gpu


def test_alphas_matches_oracle(vgx, pdf_ctx, c1_grid):
    import torch
    print("alpha_s interpolation vs oracle", flush=True)
    table = synthetic_alphas(c1_grid)
    vgx.pdf_set_alphas(pdf_ctx, table.q2_knots, table.values)
    lo, hi = table.q2_knots[0][0], table.q2_knots[-1][-1]
    rng = np.random.default_rng(5)
    q2 = np.concatenate([np.exp(rng.uniform(np.log(lo), np.log(hi), 100_003)),
                         np.concatenate(table.q2_knots),            # knots, thresholds included
                         [hi, hi * 1.0000001, hi * 50, lo, lo * 0.999, 0.5 * lo]])
    out = torch.empty(q2.size, dtype=torch.float64, device="cuda")
    vgx.pdf_alphas(pdf_ctx, torch.from_numpy(q2).cuda(), out)
    got = out.cpu().numpy()
    ref = oa.interp(table, q2)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan) and nan.sum() == 2
    assert np.allclose(got[~nan], ref[~nan], rtol=1e-13, atol=0)
    assert np.all(got[q2 > hi] == table.values[-1][-1])


def test_alphas_errors(vgx, c1_grid):
    import torch
    pdf = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    try:
        q = torch.ones(4, dtype=torch.float64, device="cuda")
        with pytest.raises(vgx.VgxError):
            vgx.pdf_alphas(pdf, q, torch.empty_like(q))  # no table attached
        with pytest.raises(vgx.VgxError):
            vgx.pdf_set_alphas(pdf, np.array([1.0, 3.0, 2.0]), np.array([0.3, 0.2, 0.25]))  # not ascending
        with pytest.raises(vgx.VgxError):
            vgx.pdf_set_alphas(pdf, np.array([1.0, 2.0, 2.0]), np.array([0.3, 0.2, 0.2]))  # 1-knot subgrid
    finally:
        vgx.pdf_destroy(pdf)

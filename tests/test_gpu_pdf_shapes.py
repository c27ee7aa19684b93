"""GPU PDF interpolation on small random grids vs the FP64 oracle: flavour
counts other than 11 (the kernels' run-time flavour count), grids of two to
nine x knots and subgrids of two to six Q^2 knots, where most or all cells
take the bilinear rule, plus exact knots, thresholds and the grid's corners.
Bars as for the full grid: FP64 output 1e-13, FP32 output 1e-5, relative or
against the largest node value (values are O(1) here)."""
import types

import numpy as np
import pytest

from oracle import pdf as opdf

pytestmark = pytest.mark.gpu

SHAPES = [  # (n_flav, n_x, knots per subgrid)
    (1, 2, [2]),
    (3, 3, [2, 3]),
    (5, 4, [4]),
    (11, 5, [2, 2, 3]),
    (13, 7, [3, 5, 2]),
    (16, 9, [6, 4]),
]


def random_grid(n_flav, n_x, nqs, seed):
    rng = np.random.default_rng(seed)
    lx = np.cumsum(rng.uniform(0.3, 1.5, n_x))
    x = np.exp(lx - lx[-1]) * 0.9  # ascending, largest 0.9, uneven spacing
    q2_knots, lo = [], 1.0
    for nq in nqs:
        q = lo * np.exp(np.concatenate([[0.0], np.cumsum(rng.uniform(0.2, 1.2, nq - 1))]))
        q2_knots.append(q)
        lo = q[-1]
    xf = [rng.uniform(-0.5, 2.0, (n_flav, len(q), n_x)) for q in q2_knots]
    return types.SimpleNamespace(x_knots=x, q2_knots=q2_knots, xf=xf, n_flav=n_flav)


def queries(grid, n, seed):
    rng = np.random.default_rng(seed)
    x0, x1 = grid.x_knots[0], grid.x_knots[-1]
    qs = np.concatenate(grid.q2_knots)
    x = np.exp(rng.uniform(np.log(x0), np.log(x1), n))
    q2 = np.exp(rng.uniform(np.log(qs[0]), np.log(qs[-1]), n))
    # knots, thresholds and corners
    ex_x = np.concatenate([grid.x_knots, [x0, x1, x0, x1]])
    ex_q = np.concatenate([rng.choice(qs, grid.x_knots.size), [qs[0], qs[0], qs[-1], qs[-1]]])
    return np.concatenate([x, ex_x]), np.concatenate([q2, ex_q])


@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_small_grids_match_oracle(vgx, shape):
    import torch
    n_flav, n_x, nqs = SHAPES[shape]
    print(f"pdf small grid n_flav={n_flav} n_x={n_x} nq={nqs}", flush=True)
    grid = random_grid(n_flav, n_x, nqs, 50 + shape)
    x, q2 = queries(grid, 3001, 60 + shape)
    ref = opdf.interp(grid, x, q2)
    scale = max(np.abs(v).max() for v in grid.xf)
    ctx = vgx.pdf_create(grid.x_knots, grid.q2_knots, grid.xf)
    try:
        xt, qt = torch.tensor(x, device="cuda"), torch.tensor(q2, device="cuda")
        for dt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-5)):
            res = torch.empty((n_flav, x.size), dtype=dt, device="cuda")
            vgx.pdf_interp(ctx, xt, qt, res)
            torch.cuda.synchronize()
            got = res.double().cpu().numpy()
            err = np.abs(got - ref)
            ok = (err <= tol * np.abs(ref)) | (err <= tol * scale)
            assert ok.all(), f"{dt}: worst error {err[~ok].max():.3e}"
        assert vgx.pdf_out_of_range(ctx) == 0
    finally:
        vgx.pdf_destroy(ctx)


def test_non_finite_grid_values_rejected(vgx):
    grid = random_grid(3, 4, [3], 7)
    for bad in (np.nan, np.inf, -np.inf, 1e39):  # 1e39 overflows the FP32 copy
        xf = [v.copy() for v in grid.xf]
        xf[0][1, 2, 3] = bad
        with pytest.raises(vgx.VgxError):
            vgx.pdf_create(grid.x_knots, grid.q2_knots, xf)
    ctx = vgx.pdf_create(grid.x_knots, grid.q2_knots, grid.xf)
    vgx.pdf_destroy(ctx)


def test_knot_count_beyond_lds_rejected(vgx):
    """The interpolation kernel keeps the knots and a slot per query of each
    wave in 64 KiB of LDS: 16 bytes per knot plus 2048 x (9 | 1) bytes for one
    flavour, so 2944 knots in all fit and 2945 do not."""
    def grid(n_x):
        x = np.exp(np.linspace(-20.0, 0.0, n_x))
        return x, [np.array([1.0, 2.0])], [np.ones((1, 2, n_x))]
    ctx = vgx.pdf_create(*grid(2942))
    vgx.pdf_destroy(ctx)
    with pytest.raises(vgx.VgxError):
        vgx.pdf_create(*grid(2943))

"""GPU log-bicubic PDF interpolation vs the FP64 oracle (through the C ABI).

Metric: the thesis's relative difference r_i = |a - b| / (|b| + eps) with
eps = 1e-16 (PDFFlow accuracy equation).  Bars: FP64 output r_i <= 1e-13,
FP32 output r_i <= 1e-5.  Where the stencil combination cancels (values
near zero next to larger node values) a relative bar is not meaningful, so
an absolute floor proportional to the largest node value of the stencil is
allowed: |a - b| <= tol * max|F_stencil|, the rounding bound of a weighted
sum whose weights have magnitude <= 1.3.
"""
import numpy as np
import pytest

from oracle import pdf as opdf
from synth import pdf_queries, C1

pytestmark = pytest.mark.gpu

EPS = 1e-16


def stencil_scale(grid, x, q2):
    """max |F| over the nodes any interpolation at (x, q2) may touch."""
    sub = opdf.find_subgrid(grid.q2_knots, q2)
    out = np.zeros(x.shape)
    for s in range(len(grid.q2_knots)):
        m = sub == s
        if not m.any():
            continue
        F = np.abs(grid.xf[s]).max(axis=0)  # (nq, nx) over flavours
        i = opdf.find_cell(grid.x_knots, x[m])
        j = opdf.find_cell(grid.q2_knots[s], q2[m])
        best = np.zeros(m.sum())
        for dr in (-1, 0, 1, 2):
            for dk in (-1, 0, 1, 2):
                jr = np.clip(j + dr, 0, F.shape[0] - 1)
                ik = np.clip(i + dk, 0, F.shape[1] - 1)
                best = np.maximum(best, F[jr, ik])
        out[m] = best
    return out


def check(got, ref, scale, tol):
    r = np.abs(got - ref) / (np.abs(ref) + EPS)
    ok = (r <= tol) | (np.abs(got - ref) <= tol * scale[None, :])
    return ok, r


@pytest.mark.parametrize("n", [1, 255, 257, 100_003])
@pytest.mark.parametrize("out", ["f64", "f32"])
def test_random_queries_match_oracle(vgx, pdf_ctx, c1_grid, n, out):
    import torch
    print(f"pdf_interp n={n} out={out}", flush=True)
    x, q2 = pdf_queries(n, seed=1000 + n)
    xt = torch.tensor(x, device="cuda")
    qt = torch.tensor(q2, device="cuda")
    dt = torch.float64 if out == "f64" else torch.float32
    res = torch.empty((11, n), dtype=dt, device="cuda")
    vgx.pdf_interp(pdf_ctx, xt, qt, res)
    torch.cuda.synchronize()
    got = res.double().cpu().numpy()
    ref = opdf.interp(c1_grid, x, q2)
    tol = 1e-13 if out == "f64" else 1e-5
    ok, r = check(got, ref, stencil_scale(c1_grid, x, q2), tol)
    assert ok.all(), f"worst r_i {r[~ok].max():.3e} at {np.argwhere(~ok)[:3]}"
    assert vgx.pdf_out_of_range(pdf_ctx) == 0


def test_full_query_range_including_lowest_subgrid_and_edges(vgx, pdf_ctx, c1_grid):
    import torch
    rng = np.random.default_rng(5)
    n = 50_000
    # x over the whole grid incl. edge (bilinear) cells; Q^2 over all subgrids
    x = np.exp(rng.uniform(np.log(1e-9), 0.0, n))
    q2 = np.exp(rng.uniform(np.log(1.0), np.log(1e10), n))
    # exact knots, thresholds and grid corners
    extra_x = np.concatenate([c1_grid.x_knots[[0, 1, 2, 97, 193, 194, 195]], [1.0, 1e-9]])
    extra_q = np.concatenate([[1.0, 1.69, 1.3 ** 2, 4.75 ** 2, 1e10, 1e10 * (1 - 1e-15)]])
    X, Q = np.meshgrid(extra_x, extra_q)
    x = np.concatenate([x, X.ravel()])
    q2 = np.concatenate([q2, Q.ravel()])
    res = torch.empty((11, len(x)), dtype=torch.float64, device="cuda")
    vgx.pdf_interp(pdf_ctx, torch.tensor(x, device="cuda"), torch.tensor(q2, device="cuda"), res)
    got = res.cpu().numpy()
    ref = opdf.interp(c1_grid, x, q2)
    ok, r = check(got, ref, stencil_scale(c1_grid, x, q2), 1e-13)
    assert ok.all()
    assert vgx.pdf_out_of_range(pdf_ctx) == 0


def test_node_values_exact(vgx, pdf_ctx, c1_grid):
    import torch
    xs, qs, refs = [], [], []
    for s, q2 in enumerate(c1_grid.q2_knots):
        for j in range(len(q2) - 1):
            for i in range(0, 196, 5):
                xs.append(c1_grid.x_knots[i]); qs.append(q2[j]); refs.append(c1_grid.xf[s][:, j, i])
    x, q2 = np.array(xs), np.array(qs)
    res = torch.empty((11, len(x)), dtype=torch.float64, device="cuda")
    vgx.pdf_interp(pdf_ctx, torch.tensor(x, device="cuda"), torch.tensor(q2, device="cuda"), res)
    assert np.allclose(res.cpu().numpy(), np.array(refs).T, rtol=1e-14, atol=0)


def test_out_of_grid_gives_nan_and_is_counted(vgx, pdf_ctx):
    import torch
    x = torch.tensor([0.5, 1e-10, 1.5, 0.1, 0.1], dtype=torch.float64, device="cuda")
    q2 = torch.tensor([100.0, 100.0, 100.0, 0.5, 2e10], dtype=torch.float64, device="cuda")
    res = torch.empty((11, 5), dtype=torch.float64, device="cuda")
    vgx.pdf_interp(pdf_ctx, x, q2, res)
    r = res.cpu().numpy()
    assert np.isfinite(r[:, 0]).all()
    assert np.isnan(r[:, 1:]).all()
    assert vgx.pdf_out_of_range(pdf_ctx) == 4
    assert vgx.pdf_out_of_range(pdf_ctx) == 0


def test_bounds_and_empty(vgx, pdf_ctx):
    import torch
    xmin, xmax, q2min, q2max = vgx.pdf_bounds(pdf_ctx)
    assert (xmin, xmax, q2min, q2max) == (1e-9, 1.0, 1.0, 1e10)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    vgx.pdf_interp(pdf_ctx, e, e, torch.empty((11, 0), dtype=torch.float64, device="cuda"))


def test_malformed_grid_rejected(vgx):
    with pytest.raises(vgx.VgxError):
        vgx.pdf_create(np.array([0.1, 0.05, 1.0]), [np.array([1.0, 2.0])], [np.zeros((1, 2, 3))])
    with pytest.raises(vgx.VgxError):
        vgx.pdf_create(np.array([0.1, 0.5, 1.0]), [np.array([1.0, 2.0]), np.array([2.5, 3.0])],
                       [np.zeros((1, 2, 3)), np.zeros((1, 2, 3))])


def test_full_size_sampled(vgx, pdf_ctx, c1_grid):
    """The benchmark launch (1e8 queries, FP32 and FP64 outputs) checked on
    a sample of outputs the oracle computes one by one."""
    import torch
    n = C1["n_queries"]
    print(f"pdf_interp full size n={n}", flush=True)
    g = torch.Generator(device="cpu").manual_seed(11)
    x, q2 = pdf_queries(n)
    xt = torch.from_numpy(x).cuda()
    qt = torch.from_numpy(q2).cuda()
    del x, q2
    idx = np.sort(np.random.default_rng(3).choice(n, 20000, replace=False))
    for dt, tol in ((torch.float32, 1e-5), (torch.float64, 1e-13)):
        res = torch.empty((11, n), dtype=dt, device="cuda")
        vgx.pdf_interp(pdf_ctx, xt, qt, res)
        it = torch.from_numpy(idx).cuda()
        got = res[:, it].double().cpu().numpy()
        xs, qs = xt[it].cpu().numpy(), qt[it].cpu().numpy()
        ref = opdf.interp(c1_grid, xs, qs)
        ok, r = check(got, ref, stencil_scale(c1_grid, xs, qs), tol)
        assert ok.all()
        del res
        torch.cuda.empty_cache()

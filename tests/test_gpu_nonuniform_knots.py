"""Fused integrands and the stand-alone interpolation on a PDF grid whose
knots are not evenly spaced in ln x or ln Q^2 (every interior knot moved by
up to +-20 % of a spacing), against the FP64 oracle on the same grid.

Real PDF sets are not evenly spaced.  On such a grid the fused integrands
leave their spacing-based cell guess for the general search over the staged
knots (fixed-scale rows: binary search; per-event scale: both axes) and the
Hermite weights use unequal neighbour spacings, so this file runs those
branches.  Bars: `tests/fp32_bars.py` (per event) and the thesis's r_i for
the stand-alone interpolation (as in `test_gpu_pdf.py`).
"""
import math

import numpy as np
import pytest

from oracle import drellyan as dy, pdf as opdf, singletop as ost, ttbar, vegas as ov
from oracle.philox import sample_uniforms
from synth import C2, C5, C6, nonuniform_pdf_grid, pdf_queries, synthetic_alphas
from tests.fp32_bars import check_events

pytestmark = pytest.mark.gpu

TT = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])
DY = np.array([C5["sqrt_s"], C5["m_lo"], C5["m_hi"], C5["m_z"], C5["gamma_z"], C5["sw2"], C5["alpha_em"],
               C5["gev2_to_pb"]])
ST = np.array([C6["sqrt_s"], C6["m_top"], C6["m_w"], C6["gamma_w"], C6["sw2"], C6["alpha_em"], C6["gev2_to_pb"]])


@pytest.fixture(scope="module")
def nu_grid():
    return nonuniform_pdf_grid()


@pytest.fixture(scope="module")
def nu_pdf(vgx, nu_grid):
    h = vgx.pdf_create(nu_grid.x_knots, nu_grid.q2_knots, nu_grid.xf)
    yield h
    vgx.pdf_destroy(h)


def near_x_knot(grid, x1, x2):
    xk = grid.x_knots
    bad = np.zeros(len(x1), dtype=bool)
    for xv in (x1, x2):
        i = np.clip(np.searchsorted(xk, xv), 1, len(xk) - 1)
        d = np.minimum(np.abs(xv - xk[i - 1]), np.abs(xv - xk[i])) / xv
        bad |= d < 1e-6
    return bad


def near_q2_knot(grid, q2):
    qk = np.concatenate(grid.q2_knots)
    i = np.clip(np.searchsorted(qk, q2), 1, len(qk) - 1)
    return np.minimum(np.abs(q2 - qk[i - 1]), np.abs(q2 - qk[i])) / q2 < 1e-6


def sample_on_gpu(vgx, v, n, it, grid_kind, n_bins):
    import torch
    if grid_kind == "adapted":
        for k in range(3):
            vgx.vegas_iterate(v, 200_000, k)
            vgx.vegas_refine(v)
    e = vgx.vegas_get_grid(v, 3, n_bins)
    g = torch.empty(n, dtype=torch.float64, device="cuda")
    vgx.vegas_sample(v, 0, n, it, g=g)
    return g.cpu().numpy(), e


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("grid_kind", ["uniform", "adapted"])
def test_ttbar_fixed_scale_per_event(vgx, nu_pdf, nu_grid, grid_kind, mode):
    print(f"non-uniform knots: ttbar per-event, {grid_kind} grid, mode {mode}", flush=True)
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], C2["seed"], 0, vgx.F32,
                         np.concatenate([TT, [float(mode)]]), pdf=nu_pdf)
    try:
        n = 50_000
        got, e = sample_on_gpu(vgx, v, n, 9, grid_kind, C2["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(C2["seed"], 0, 9, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, e)
    ref = ttbar.integrand(x, nu_grid, C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]) * jac
    k = ttbar.phase_space(x, C2["sqrt_s"], C2["m_top"])
    keep = ~near_x_knot(nu_grid, k["x1"], k["x2"])
    assert keep.sum() > 0.999 * n
    check_events(got, ref, keep, f"ttbar mode {mode} {grid_kind}")


@pytest.mark.parametrize("grid_kind", ["uniform", "adapted"])
def test_ttbar_scale_per_event(vgx, nu_pdf, nu_grid, grid_kind):
    """mu^2 = s_hat/4 and alpha_s(mu) per event: both the x and the Q^2 cell
    searches take the general path (the alpha_s knots are the grid's Q^2
    knots, so they are uneven too)."""
    print(f"non-uniform knots: ttbar mode 2 per-event, {grid_kind} grid", flush=True)
    table = synthetic_alphas(nu_grid)
    vgx.pdf_set_alphas(nu_pdf, table.q2_knots, table.values)
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], C2["seed"], 0, vgx.F32,
                         np.concatenate([TT, [2.0]]), pdf=nu_pdf)
    try:
        n = 50_000
        got, e = sample_on_gpu(vgx, v, n, 9, grid_kind, C2["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(C2["seed"], 0, 9, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, e)
    ref = ttbar.integrand_dynamic(x, nu_grid, table, C2["sqrt_s"], C2["m_top"], C2["gev2_to_pb"]) * jac
    k = ttbar.phase_space(x, C2["sqrt_s"], C2["m_top"])
    keep = ~(near_x_knot(nu_grid, k["x1"], k["x2"]) | near_q2_knot(nu_grid, k["shat"] / 4))
    assert keep.sum() > 0.999 * n
    check_events(got, ref, keep, f"ttbar mode 2 {grid_kind}")


@pytest.mark.parametrize("mode", [0, 1])
def test_drell_yan_per_event(vgx, nu_pdf, nu_grid, mode):
    print(f"non-uniform knots: drell-yan per-event, mode {mode}", flush=True)
    v = vgx.vegas_create(vgx.DRELLYAN, 3, C5["n_bins"], C5["alpha"], C5["seed"], 0, vgx.F32,
                         np.concatenate([DY, [float(mode)]]), pdf=nu_pdf)
    try:
        n = 50_000
        got, e = sample_on_gpu(vgx, v, n, 9, "adapted", C5["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(C5["seed"], 0, 9, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, e)
    ref = dy.integrand_from_config(x, nu_grid, C5) * jac
    k = dy.phase_space(x, C5["sqrt_s"], C5["m_lo"], C5["m_hi"])
    keep = ~near_x_knot(nu_grid, k["x1"], k["x2"])
    assert keep.sum() > 0.999 * n
    check_events(got, ref, keep, f"drell-yan mode {mode}")


@pytest.mark.parametrize("mode", [0, 1])
def test_single_top_per_event(vgx, nu_pdf, nu_grid, mode):
    print(f"non-uniform knots: single top per-event, mode {mode}", flush=True)
    v = vgx.vegas_create(vgx.SINGLETOP, 3, C6["n_bins"], C6["alpha"], C6["seed"], 0, vgx.F32,
                         np.concatenate([ST, [float(mode)]]), pdf=nu_pdf)
    try:
        n = 50_000
        got, e = sample_on_gpu(vgx, v, n, 9, "adapted", C6["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(C6["seed"], 0, 9, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, e)
    ref = ost.integrand_from_config(x, nu_grid, C6) * jac
    k = ost.phase_space(x, C6["sqrt_s"], C6["m_top"])
    keep = ~near_x_knot(nu_grid, k["x1"], k["x2"])
    assert keep.sum() > 0.999 * n
    check_events(got, ref, keep, f"single top mode {mode}")


def test_ttbar_full_size_iteration(vgx, nu_pdf, nu_grid):
    """The benchmark's launch shape (1e7 events) on the uneven grid: sums and
    histogram against the oracle over every event."""
    print("non-uniform knots: ttbar full-size 1e7 vs oracle", flush=True)
    n = C2["n_per_iter"]
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], C2["seed"], 0, vgx.F32,
                         np.concatenate([TT, [0.0]]), pdf=nu_pdf)
    try:
        for it in range(2):
            vgx.vegas_iterate(v, 1_000_000, it)
            vgx.vegas_refine(v)
        e = vgx.vegas_get_grid(v, 3, C2["n_bins"])
        r = vgx.vegas_iterate(v, n, 5)
        h = vgx.vegas_get_hist(v, 3, C2["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    p1, p2 = [], []
    hist = np.zeros((3, C2["n_bins"]))
    for first in range(0, n, 1_000_000):
        idx = np.arange(first, min(first + 1_000_000, n), dtype=np.uint64)
        u = sample_uniforms(C2["seed"], 0, 5, idx, 3)
        x, jac, bins = ov.vegas_map(u, e)
        w = ttbar.integrand(x, nu_grid, C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]) * jac
        p1.append(math.fsum(w))
        p2.append(math.fsum(w * w))
        for j in range(3):
            hist[j] += np.bincount(bins[:, j], weights=w * w, minlength=C2["n_bins"])
    s1, s2 = math.fsum(p1), math.fsum(p2)
    print(f"  S1 rel {abs(r['s1'] - s1) / abs(s1):.2e}, S2 rel {abs(r['s2'] - s2) / abs(s2):.2e}", flush=True)
    assert r["s1"] == pytest.approx(s1, rel=1e-5)
    assert r["s2"] == pytest.approx(s2, rel=2e-5)
    assert np.allclose(h, hist, rtol=2e-5, atol=1e-6 * hist.sum() / 3)


@pytest.mark.parametrize("out", ["f64", "f32"])
def test_standalone_interpolation(vgx, nu_pdf, nu_grid, out):
    import torch
    from tests.test_gpu_pdf import check, stencil_scale
    print(f"non-uniform knots: pdf_interp out={out}", flush=True)
    n = 100_003
    x, q2 = pdf_queries(n, seed=77)
    res = torch.empty((11, n), dtype=torch.float64 if out == "f64" else torch.float32, device="cuda")
    vgx.pdf_interp(nu_pdf, torch.tensor(x, device="cuda"), torch.tensor(q2, device="cuda"), res)
    got = res.double().cpu().numpy()
    ref = opdf.interp(nu_grid, x, q2)
    tol = 1e-13 if out == "f64" else 1e-5
    ok, r = check(got, ref, stencil_scale(nu_grid, x, q2), tol)
    print(f"  r_i max {r.max():.2e} p99 {np.percentile(r, 99):.2e}", flush=True)
    assert ok.all()

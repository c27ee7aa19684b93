"""GPU fused t tbar integrand (FP32 integrand, FP64 map and sums) vs oracle.

Per-event bars and their error model: `tests/fp32_bars.py` (relative 1e-5,
also at the 99th percentile; an absolute floor of 1e-7 of the mean weight
for at most 0.5 % of the events, those with tiny cancelling luminosities).
Events whose x lies within 1e-6 (relative) of a knot may be assigned the
neighbouring cell by the FP32 search; the interpolant is continuous there
except at the bicubic/bilinear switch of the last x cell, so those events
are excluded and counted.
"""
import math

import numpy as np
import pytest

from oracle import ttbar, vegas as ov
from oracle.philox import sample_uniforms
from synth import C2
from tests.fp32_bars import check_events

pytestmark = pytest.mark.gpu

PARAMS = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])


def make(vgx, pdf_ctx, seed=C2["seed"], mode=0):
    params = np.concatenate([PARAMS, [float(mode)]])
    return vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], seed, 0, vgx.F32, params, pdf=pdf_ctx)


def near_knot(grid, u):
    k = ttbar.phase_space(u, C2["sqrt_s"], C2["m_top"])
    xk = grid.x_knots
    bad = np.zeros(len(u), dtype=bool)
    for xv in (k["x1"], k["x2"]):
        i = np.clip(np.searchsorted(xk, xv), 1, len(xk) - 1)
        d = np.minimum(np.abs(xv - xk[i - 1]), np.abs(xv - xk[i])) / xv
        bad |= d < 1e-6
    return bad


def oracle_g(grid, u, e):
    x, jac, _ = ov.vegas_map(u, e)
    return ttbar.integrand(x, grid, C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]) * jac, x


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("grid_kind", ["uniform", "adapted"])
def test_per_event_integrand(vgx, pdf_ctx, c1_grid, grid_kind, mode):
    """mode 0: full (ln x, ln Q^2) stencil per event; mode 1: the Q^2
    direction contracted once at the fixed scale (same interpolant)."""
    import torch
    print(f"ttbar per-event, {grid_kind} grid, mode {mode}", flush=True)
    v = make(vgx, pdf_ctx, mode=mode)
    try:
        if grid_kind == "adapted":
            for it in range(3):
                vgx.vegas_iterate(v, 200_000, it)
                vgx.vegas_refine(v)
        e = vgx.vegas_get_grid(v, 3, C2["n_bins"])
        n = 50_000
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.vegas_sample(v, 0, n, 9, g=g)
        got = g.cpu().numpy()
        u = sample_uniforms(C2["seed"], 0, 9, np.arange(n, dtype=np.uint64), 3)
        ref, x = oracle_g(c1_grid, u, e)
        keep = ~near_knot(c1_grid, x)
        assert keep.sum() > 0.999 * n
        check_events(got, ref, keep, f"ttbar mode {mode} {grid_kind}")
    finally:
        vgx.vegas_destroy(v)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("sqrt_s,m_top", [(2000.0, 172.5), (7000.0, 173.0), (100000.0, 173.0)])
def test_per_event_integrand_other_energies(vgx, pdf_ctx, c1_grid, sqrt_s, m_top, mode):
    """Other collider energies and top masses move the smallest reachable
    momentum fraction tau0 = 4 m^2/s, hence how many x nodes the context
    stages (about 30 at 2 TeV, 130 at 100 TeV) and the size of the tables
    every workgroup copies; per event against the oracle."""
    import torch
    print(f"ttbar per-event at sqrt_s={sqrt_s} m_t={m_top}, mode {mode}", flush=True)
    params = np.array([sqrt_s, m_top, C2["alpha_s"], C2["gev2_to_pb"], float(mode)])
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], 5, 0, vgx.F32, params, pdf=pdf_ctx)
    try:
        n = 40_000
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.vegas_sample(v, 0, n, 2, g=g)
        got = g.cpu().numpy()
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(5, 0, 2, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, ov.uniform_grid(3, C2["n_bins"]))
    ref = ttbar.integrand(x, c1_grid, sqrt_s, m_top, C2["alpha_s"], C2["gev2_to_pb"]) * jac
    k = ttbar.phase_space(x, sqrt_s, m_top)
    xk = c1_grid.x_knots
    keep = np.ones(n, dtype=bool)
    for xv in (k["x1"], k["x2"]):
        i = np.clip(np.searchsorted(xk, xv), 1, len(xk) - 1)
        keep &= np.minimum(np.abs(xv - xk[i - 1]), np.abs(xv - xk[i])) / xv >= 1e-6
    assert keep.sum() > 0.999 * n
    check_events(got, ref, keep, f"ttbar sqrt_s={sqrt_s} mode {mode}")


def test_iteration_sums(vgx, pdf_ctx, c1_grid):
    print("ttbar one iteration 2e5", flush=True)
    v = make(vgx, pdf_ctx)
    try:
        n = 200_000
        r = vgx.vegas_iterate(v, n, 0)
        u = sample_uniforms(C2["seed"], 0, 0, np.arange(n, dtype=np.uint64), 3)
        e = ov.uniform_grid(3, C2["n_bins"])
        ref, _ = oracle_g(c1_grid, u, e)
        # FP32 integrand, FP64 sums: the sums inherit the per-event 1e-5 bar
        assert r["s1"] == pytest.approx(math.fsum(ref), rel=1e-5)
        assert r["s2"] == pytest.approx(math.fsum(ref * ref), rel=2e-5)
        h = vgx.vegas_get_hist(v, 3, C2["n_bins"])
        _, _, idx = ov.vegas_map(u, e)
        for j in range(3):
            hj = np.bincount(idx[:, j], weights=ref * ref, minlength=C2["n_bins"])
            assert np.allclose(h[j], hj, rtol=2e-5, atol=1e-6 * hj.sum())
    finally:
        vgx.vegas_destroy(v)


def test_full_run_against_quadrature(vgx, pdf_ctx, c1_grid):
    """Ten iterations of 1e6 events; the result must agree with the 2-d
    quadrature of the closed-form partonic cross sections."""
    print("ttbar 10 x 1e6 vs quadrature", flush=True)
    from tests.test_oracle_ttbar import _lumi_sigma
    v = make(vgx, pdf_ctx)
    try:
        for it in range(10):
            vgx.vegas_iterate(v, 1_000_000, it)
            vgx.vegas_refine(v)
        res = vgx.vegas_result(v)
    finally:
        vgx.vegas_destroy(v)
    xg, wg = np.polynomial.legendre.leggauss(120)
    uu, ww = 0.5 * (xg + 1), 0.5 * wg
    s = C2["sqrt_s"] ** 2
    tau0 = 4 * C2["m_top"] ** 2 / s
    total = 0.0
    for u1, w1 in zip(uu, ww):
        tau = tau0 ** (1 - u1)
        jt = tau * math.log(1 / tau0)
        ly = math.log(1 / tau)
        for u2, w2 in zip(uu, ww):
            total += w1 * w2 * jt * ly * _lumi_sigma(c1_grid, tau, (u2 - 0.5) * ly)
    assert abs(res["mean"] - total) < 4 * res["sigma"] + 2e-5 * total
    assert res["sigma"] / res["mean"] < 2e-3


def test_full_size_iteration_matches_oracle(vgx, pdf_ctx, c1_grid):
    """The benchmark launch (1e7 events, same kernel and launch shape) against
    the oracle over all 1e7 events (computed in chunks): the sums to the
    per-event bar, the histogram to 2e-5."""
    print("ttbar full-size 1e7 vs oracle", flush=True)
    n = C2["n_per_iter"]
    v = make(vgx, pdf_ctx)
    try:
        for it in range(2):          # an adapted grid for the measured iteration
            vgx.vegas_iterate(v, 1_000_000, it)
            vgx.vegas_refine(v)
        e = vgx.vegas_get_grid(v, 3, C2["n_bins"])
        r = vgx.vegas_iterate(v, n, 5)
        h = vgx.vegas_get_hist(v, 3, C2["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    parts1, parts2 = [], []
    hist = np.zeros((3, C2["n_bins"]))
    chunk = 1_000_000
    for first in range(0, n, chunk):
        idx = np.arange(first, min(first + chunk, n), dtype=np.uint64)
        u = sample_uniforms(C2["seed"], 0, 5, idx, 3)
        w, _ = oracle_g(c1_grid, u, e)
        parts1.append(math.fsum(w))
        parts2.append(math.fsum(w * w))
        _, _, bins = ov.vegas_map(u, e)
        for j in range(3):
            hist[j] += np.bincount(bins[:, j], weights=w * w, minlength=C2["n_bins"])
    assert r["s1"] == pytest.approx(math.fsum(parts1), rel=1e-5)
    assert r["s2"] == pytest.approx(math.fsum(parts2), rel=2e-5)
    assert np.allclose(h, hist, rtol=2e-5, atol=1e-6 * hist.sum() / 3)


# --- scale set per event (mode 2): mu^2 = s_hat/4, alpha_s(mu) from the table


def make_dyn(vgx, pdf_ctx, c1_grid, seed=C2["seed"]):
    from synth import synthetic_alphas
    table = synthetic_alphas(c1_grid)
    vgx.pdf_set_alphas(pdf_ctx, table.q2_knots, table.values)
    params = np.concatenate([PARAMS, [2.0]])
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], seed, 0, vgx.F32, params, pdf=pdf_ctx)
    return v, table


def near_knot_dyn(grid, x):
    """Events within 1e-6 (relative) of an x knot or of a Q^2 knot at their
    scale: the FP32 cell search may pick the neighbouring cell there."""
    bad = near_knot(grid, x)
    k = ttbar.phase_space(x, C2["sqrt_s"], C2["m_top"])
    qk = np.concatenate(grid.q2_knots)
    mu2 = k["shat"] / 4
    i = np.clip(np.searchsorted(qk, mu2), 1, len(qk) - 1)
    d = np.minimum(np.abs(mu2 - qk[i - 1]), np.abs(mu2 - qk[i])) / mu2
    return bad | (d < 1e-6)


@pytest.mark.parametrize("grid_kind", ["uniform", "adapted"])
def test_dynamic_scale_per_event(vgx, pdf_ctx, c1_grid, grid_kind):
    import torch
    print(f"ttbar mode 2 per-event, {grid_kind} grid", flush=True)
    v, table = make_dyn(vgx, pdf_ctx, c1_grid)
    try:
        if grid_kind == "adapted":
            for it in range(3):
                vgx.vegas_iterate(v, 200_000, it)
                vgx.vegas_refine(v)
        e = vgx.vegas_get_grid(v, 3, C2["n_bins"])
        n = 50_000
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.vegas_sample(v, 0, n, 9, g=g)
        got = g.cpu().numpy()
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(C2["seed"], 0, 9, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, e)
    ref = ttbar.integrand_dynamic(x, c1_grid, table, C2["sqrt_s"], C2["m_top"], C2["gev2_to_pb"]) * jac
    keep = ~near_knot_dyn(c1_grid, x)
    assert keep.sum() > 0.999 * n
    check_events(got, ref, keep, f"ttbar mode 2 {grid_kind}")


def test_dynamic_scale_iteration_and_quadrature(vgx, pdf_ctx, c1_grid):
    """One 2e5 iteration against the oracle's sums, then ten iterations of 1e6
    against the quadrature with alpha_s and PDFs at mu^2 = s_hat/4."""
    print("ttbar mode 2 sums and 10 x 1e6 vs quadrature", flush=True)
    from tests.test_oracle_ttbar import dynamic_scale_quadrature
    v, table = make_dyn(vgx, pdf_ctx, c1_grid)
    try:
        n = 200_000
        r = vgx.vegas_iterate(v, n, 0)
        vgx.vegas_refine(v)
        for it in range(1, 10):
            vgx.vegas_iterate(v, 1_000_000, it)
            vgx.vegas_refine(v)
        res = vgx.vegas_result(v)
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(C2["seed"], 0, 0, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, ov.uniform_grid(3, C2["n_bins"]))
    w = ttbar.integrand_dynamic(x, c1_grid, table, C2["sqrt_s"], C2["m_top"], C2["gev2_to_pb"]) * jac
    assert r["s1"] == pytest.approx(math.fsum(w), rel=1e-5)
    assert r["s2"] == pytest.approx(math.fsum(w * w), rel=2e-5)
    total = dynamic_scale_quadrature(c1_grid, table)
    assert abs(res["mean"] - total) < 4 * res["sigma"] + 2e-5 * total
    assert res["sigma"] / res["mean"] < 2e-3


@pytest.mark.parametrize("sqrt_s", [7000.0, 100000.0])
def test_dynamic_scale_per_event_other_energies(vgx, pdf_ctx, c1_grid, sqrt_s):
    """The per-event scale spans [m_t^2, s/4]: other energies change how many
    Q^2 rows the context stages (about 10 at 7 TeV, 30 at 100 TeV) besides the
    x nodes; per event against the oracle."""
    import torch
    from synth import synthetic_alphas
    print(f"ttbar mode 2 per-event at sqrt_s={sqrt_s}", flush=True)
    table = synthetic_alphas(c1_grid)
    vgx.pdf_set_alphas(pdf_ctx, table.q2_knots, table.values)
    params = np.array([sqrt_s, C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"], 2.0])
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], 4, 0, vgx.F32, params, pdf=pdf_ctx)
    try:
        n = 40_000
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.vegas_sample(v, 0, n, 3, g=g)
        got = g.cpu().numpy()
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(4, 0, 3, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, ov.uniform_grid(3, C2["n_bins"]))
    ref = ttbar.integrand_dynamic(x, c1_grid, table, sqrt_s, C2["m_top"], C2["gev2_to_pb"]) * jac
    k = ttbar.phase_space(x, sqrt_s, C2["m_top"])
    xk = c1_grid.x_knots
    qk = np.concatenate(c1_grid.q2_knots)
    keep = np.ones(n, dtype=bool)
    for xv in (k["x1"], k["x2"]):
        i = np.clip(np.searchsorted(xk, xv), 1, len(xk) - 1)
        keep &= np.minimum(np.abs(xv - xk[i - 1]), np.abs(xv - xk[i])) / xv >= 1e-6
    mu2 = k["shat"] / 4
    i = np.clip(np.searchsorted(qk, mu2), 1, len(qk) - 1)
    keep &= np.minimum(np.abs(mu2 - qk[i - 1]), np.abs(mu2 - qk[i])) / mu2 >= 1e-6
    assert keep.sum() > 0.999 * n
    check_events(got, ref, keep, f"ttbar mode 2 sqrt_s={sqrt_s}")


def test_dynamic_scale_needs_alphas(vgx, c1_grid):
    pdf = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    try:
        with pytest.raises(vgx.VgxError):
            vgx.vegas_create(vgx.TTBAR, 3, 50, 1.5, 1, 0, vgx.F32, np.concatenate([PARAMS, [2.0]]), pdf=pdf)
    finally:
        vgx.pdf_destroy(pdf)


def test_dynamic_scale_context_keeps_its_tables(vgx, c1_grid):
    """A context takes the PDF rows and the alpha_s table into its staged
    tables once, at creation: replacing the PDF's alpha_s table afterwards
    leaves its iterations bit for bit as they were, while a context created
    after the change sees the new table."""
    from synth import synthetic_alphas
    print("ttbar mode 2: tables taken at creation", flush=True)
    table = synthetic_alphas(c1_grid)
    pdf = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    params = np.concatenate([PARAMS, [2.0]])
    mk = lambda: vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], C2["seed"], 0, vgx.F32, params, pdf=pdf)
    v = w = None
    try:
        vgx.pdf_set_alphas(pdf, table.q2_knots, table.values)
        v = mk()
        r0 = vgx.vegas_iterate(v, 100_000, 0)
        vgx.pdf_set_alphas(pdf, table.q2_knots, [1.1 * np.asarray(a) for a in table.values])
        r1 = vgx.vegas_iterate(v, 100_000, 0)
        w = mk()
        r2 = vgx.vegas_iterate(w, 100_000, 0)
        assert r1["s1"] == r0["s1"] and r1["s2"] == r0["s2"]
        # |M|^2 goes as alpha_s^2: the new context's estimate moves by about 1.21
        assert r2["mean"] == pytest.approx(1.21 * r0["mean"], rel=1e-4)
    finally:
        for c in (v, w):
            if c is not None:
                vgx.vegas_destroy(c)
        vgx.pdf_destroy(pdf)

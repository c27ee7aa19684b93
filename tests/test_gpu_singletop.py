"""GPU fused s-channel single-top integrand (u dbar -> t bbar; FP32
integrand, FP64 map and sums) vs the oracle.

Same bars as the t tbar integrand, for the same reasons: per event a
relative 1e-5, or an absolute error below 1e-7 of the mean weight (events
with a tiny, cancelling luminosity); events whose x lies within 1e-6
(relative) of a knot may be assigned the neighbouring cell by the FP32
search and are excluded and counted.
"""
import math

import numpy as np
import pytest

from oracle import singletop as st, vegas as ov
from oracle.philox import sample_uniforms
from synth import C6

from tests import fp32_bars

pytestmark = pytest.mark.gpu

LABEL = "single top"
PARAMS = np.array([C6["sqrt_s"], C6["m_top"], C6["m_w"], C6["gamma_w"], C6["sw2"], C6["alpha_em"],
                   C6["gev2_to_pb"]])


def make(vgx, pdf_ctx, seed=C6["seed"], mode=0):
    params = np.concatenate([PARAMS, [float(mode)]])
    return vgx.vegas_create(vgx.SINGLETOP, 3, C6["n_bins"], C6["alpha"], seed, 0, vgx.F32, params, pdf=pdf_ctx)


def near_knot(grid, x):
    k = st.phase_space(x, C6["sqrt_s"], C6["m_top"])
    xk = grid.x_knots
    bad = np.zeros(len(x), dtype=bool)
    for xv in (k["x1"], k["x2"]):
        i = np.clip(np.searchsorted(xk, xv), 1, len(xk) - 1)
        d = np.minimum(np.abs(xv - xk[i - 1]), np.abs(xv - xk[i])) / xv
        bad |= d < 1e-6
    return bad


def oracle_g(grid, u, e):
    x, jac, _ = ov.vegas_map(u, e)
    return st.integrand_from_config(x, grid, C6) * jac, x


def check_events(got, ref, keep, label="single top"):
    """Per-event bars and their error model: `tests/fp32_bars.py`."""
    return fp32_bars.check_events(got, ref, keep, label)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("grid_kind", ["uniform", "adapted"])
def test_per_event_integrand(vgx, pdf_ctx, c1_grid, grid_kind, mode):
    import torch
    print(f"single-top per-event, {grid_kind} grid, mode {mode}", flush=True)
    v = make(vgx, pdf_ctx, mode=mode)
    try:
        if grid_kind == "adapted":
            for it in range(3):
                vgx.vegas_iterate(v, 200_000, it)
                vgx.vegas_refine(v)
        e = vgx.vegas_get_grid(v, 3, C6["n_bins"])
        n = 50_000
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.vegas_sample(v, 0, n, 9, g=g)
        u = sample_uniforms(C6["seed"], 0, 9, np.arange(n, dtype=np.uint64), 3)
        ref, x = oracle_g(c1_grid, u, e)
        keep = ~near_knot(c1_grid, x)
        assert keep.sum() > 0.999 * n
        check_events(g.cpu().numpy(), ref, keep, f"{LABEL} mode {mode} {grid_kind}")
    finally:
        vgx.vegas_destroy(v)


def test_iteration_sums_and_histogram(vgx, pdf_ctx, c1_grid):
    print("single-top one iteration 2e5", flush=True)
    v = make(vgx, pdf_ctx)
    try:
        n = 200_000
        r = vgx.vegas_iterate(v, n, 0)
        h = vgx.vegas_get_hist(v, 3, C6["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(C6["seed"], 0, 0, np.arange(n, dtype=np.uint64), 3)
    e = ov.uniform_grid(3, C6["n_bins"])
    ref, _ = oracle_g(c1_grid, u, e)
    assert r["s1"] == pytest.approx(math.fsum(ref), rel=1e-5)
    assert r["s2"] == pytest.approx(math.fsum(ref * ref), rel=2e-5)
    _, _, idx = ov.vegas_map(u, e)
    for j in range(3):
        hj = np.bincount(idx[:, j], weights=ref * ref, minlength=C6["n_bins"])
        assert np.allclose(h[j], hj, rtol=2e-5, atol=1e-6 * hj.sum())


def test_full_run_against_quadrature(vgx, pdf_ctx, c1_grid):
    """Ten iterations of 1e6 events against the quadrature in ln tau of the
    luminosity times the textbook partonic cross section."""
    print("single-top 10 x 1e6 vs quadrature", flush=True)
    from scipy.integrate import quad
    from oracle.pdf import interp
    from oracle.ttbar import IDX
    v = make(vgx, pdf_ctx)
    try:
        for it in range(10):
            vgx.vegas_iterate(v, 1_000_000, it)
            vgx.vegas_refine(v)
        res = vgx.vegas_result(v)
    finally:
        vgx.vegas_destroy(v)
    s = C6["sqrt_s"] ** 2
    mt, mw, gw, sw2, al = C6["m_top"], C6["m_w"], C6["gamma_w"], C6["sw2"], C6["alpha_em"]
    xg, wg = np.polynomial.legendre.leggauss(48)

    def sig(sh):
        return math.pi * al**2 / (24 * sw2**2) * (sh - mt * mt) ** 2 * (2 * sh + mt * mt) / (
            sh * sh * ((sh - mw * mw) ** 2 + (mw * gw) ** 2))

    def dsig(lt):
        tau = math.exp(lt)
        ly = math.log(1 / tau)
        ys = 0.5 * ly * xg
        x1, x2 = math.sqrt(tau) * np.exp(ys), math.sqrt(tau) * np.exp(-ys)
        f1 = interp(c1_grid, x1, np.full(x1.shape, mt * mt))
        f2 = interp(c1_grid, x2, np.full(x2.shape, mt * mt))
        lum = sum(0.5 * ly * np.sum(wg * (f1[IDX[q]] * f2[IDX[qb]] + f1[IDX[qb]] * f2[IDX[q]]))
                  for q, qb in ((2, -1), (4, -3)))
        return lum * sig(tau * s) * C6["gev2_to_pb"]

    total, _ = quad(dsig, math.log(mt * mt / s), 0.0, epsabs=0, epsrel=1e-9, limit=200)
    assert abs(res["mean"] - total) < 4 * res["sigma"] + 2e-5 * total
    assert res["sigma"] / res["mean"] < 2e-3


def test_large_iteration_matches_oracle(vgx, pdf_ctx, c1_grid):
    """A 2e6-event iteration on an adapted grid (the benchmark's kernel and
    launch shape) against the oracle over every event."""
    print("single-top 2e6 adapted iteration vs oracle", flush=True)
    n = 2_000_000
    v = make(vgx, pdf_ctx)
    try:
        for it in range(2):
            vgx.vegas_iterate(v, 1_000_000, it)
            vgx.vegas_refine(v)
        e = vgx.vegas_get_grid(v, 3, C6["n_bins"])
        r = vgx.vegas_iterate(v, n, 5)
        h = vgx.vegas_get_hist(v, 3, C6["n_bins"])
    finally:
        vgx.vegas_destroy(v)
    p1, p2 = [], []
    hist = np.zeros((3, C6["n_bins"]))
    for first in range(0, n, 500_000):
        idx = np.arange(first, min(first + 500_000, n), dtype=np.uint64)
        u = sample_uniforms(C6["seed"], 0, 5, idx, 3)
        w, _ = oracle_g(c1_grid, u, e)
        p1.append(math.fsum(w))
        p2.append(math.fsum(w * w))
        _, _, bins = ov.vegas_map(u, e)
        for j in range(3):
            hist[j] += np.bincount(bins[:, j], weights=w * w, minlength=C6["n_bins"])
    assert r["s1"] == pytest.approx(math.fsum(p1), rel=1e-5)
    assert r["s2"] == pytest.approx(math.fsum(p2), rel=2e-5)
    assert np.allclose(h, hist, rtol=2e-5, atol=1e-6 * hist.sum() / 3)


def test_rejects_bad_parameters(vgx, pdf_ctx):
    bad = PARAMS.copy()
    bad[0] = bad[1] * 0.5  # sqrt_s below m_top
    with pytest.raises(vgx.VgxError):
        vgx.vegas_create(vgx.SINGLETOP, 3, C6["n_bins"], C6["alpha"], 1, 0, vgx.F32, bad, pdf=pdf_ctx)
    with pytest.raises(vgx.VgxError):
        vgx.vegas_create(vgx.SINGLETOP, 2, C6["n_bins"], C6["alpha"], 1, 0, vgx.F32, PARAMS, pdf=pdf_ctx)


@pytest.mark.parametrize("sqrt_s", [1960.0, 13000.0, 100000.0])
def test_per_event_integrand_other_energies(vgx, pdf_ctx, c1_grid, sqrt_s):
    """Other collider energies move the smallest reachable momentum fraction
    (m_t/sqrt s)^2, hence the x nodes the context stages; per event against
    the oracle."""
    import torch
    print(f"single top per-event at sqrt_s={sqrt_s}", flush=True)
    c = dict(C6, sqrt_s=sqrt_s)
    params = np.array([sqrt_s, c["m_top"], c["m_w"], c["gamma_w"], c["sw2"], c["alpha_em"], c["gev2_to_pb"], 0.0])
    v = vgx.vegas_create(vgx.SINGLETOP, 3, C6["n_bins"], C6["alpha"], 8, 0, vgx.F32, params, pdf=pdf_ctx)
    try:
        n = 40_000
        g = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.vegas_sample(v, 0, n, 1, g=g)
        got = g.cpu().numpy()
    finally:
        vgx.vegas_destroy(v)
    u = sample_uniforms(8, 0, 1, np.arange(n, dtype=np.uint64), 3)
    x, jac, _ = ov.vegas_map(u, ov.uniform_grid(3, C6["n_bins"]))
    ref = st.integrand_from_config(x, c1_grid, c) * jac
    k = st.phase_space(x, sqrt_s, c["m_top"])
    xk = c1_grid.x_knots
    keep = np.ones(n, dtype=bool)
    for xv in (k["x1"], k["x2"]):
        i = np.clip(np.searchsorted(xk, xv), 1, len(xk) - 1)
        keep &= np.minimum(np.abs(xv - xk[i - 1]), np.abs(xv - xk[i])) / xv >= 1e-6
    assert keep.sum() > 0.999 * n
    fp32_bars.check_events(got, ref, keep, f"single top sqrt_s={sqrt_s}")

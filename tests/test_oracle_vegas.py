"""Pins of the oracle's VEGAS map, estimator, combination and refinement."""
import math

import numpy as np
import pytest
from scipy.special import erf, ndtri

from oracle import vegas
from oracle.integrands import gauss, gauss_integral
from oracle.philox import sample_uniforms
from synth import C0


def test_gauss_closed_form_value():
    # [erf(0.5/(0.1 sqrt 2))]^4, each Gaussian factor normalised on R
    assert gauss_integral(4, 0.5, 0.1) == pytest.approx(0.99999770678939714497, rel=1e-15)
    assert gauss_integral(1, 0.3, 0.2) == pytest.approx(
        0.5 * (erf(0.7 / (0.2 * math.sqrt(2))) + erf(0.3 / (0.2 * math.sqrt(2)))), rel=1e-15)


def test_map_uniform_grid_is_identity():
    u = np.random.default_rng(0).uniform(size=(1000, 3))
    x, jac, _ = vegas.vegas_map(u, vegas.uniform_grid(3, 50))
    assert np.allclose(x, u, rtol=0, atol=1e-15)
    assert np.allclose(jac, 1.0, rtol=1e-14)


def test_map_hand_example():
    edges = np.array([[0.0, 0.2, 1.0]])
    x, jac, idx = vegas.vegas_map(np.array([[0.25], [0.75]]), edges)
    assert x[:, 0] == pytest.approx([0.1, 0.6], rel=2e-16)
    assert jac == pytest.approx([0.4, 1.6], rel=1e-15)
    assert list(idx[:, 0]) == [0, 1]


def test_map_jacobian_lattice_average_is_one():
    # On the lattice u = (k + 1/2)/M with M a multiple of N, every bin holds
    # M/N points, so mean J = sum_i width_i = 1 for any grid.
    rng = np.random.default_rng(1)
    nb, M = 50, 5000
    w = rng.uniform(0.1, 1.0, nb)
    e = np.concatenate([[0.0], np.cumsum(w) / w.sum()])
    e[-1] = 1.0
    u = ((np.arange(M) + 0.5) / M)[:, None]
    x, jac, _ = vegas.vegas_map(u, e[None, :])
    assert jac.mean() == pytest.approx(1.0, rel=1e-13)
    assert np.all(np.diff(x[:, 0]) > 0)


def test_combine_rules():
    m, s, c = vegas.combine([1.0, 3.0], [1.0, 1.0])
    assert (m, s, c) == (2.0, math.sqrt(0.5), 2.0)
    m, s, c = vegas.combine([1.0, 2.0], [1.0, 4.0])
    assert m == pytest.approx((1.0 + 2.0 / 4) / (1 + 0.25))
    assert s == pytest.approx(1 / math.sqrt(1.25))
    assert vegas.combine([5.0, 1.0], [0.0, 1.0]) == (5.0, 0.0, 0.0)


def test_mean_var_definition():
    w = np.array([1.0, 2.0, 4.0])
    mean, var = vegas.mean_var(w.sum(), (w * w).sum(), 3)
    assert mean == pytest.approx(7 / 3)
    assert var == pytest.approx(np.var(w, ddof=1) / 3)  # unbiased variance of the mean


def test_refine_constant_histogram_keeps_grid():
    rng = np.random.default_rng(2)
    w = rng.uniform(0.1, 1.0, 50)
    e = np.concatenate([[0.0], np.cumsum(w) / w.sum()])
    e[-1] = 1.0
    new = vegas.refine(e[None, :], np.full((1, 50), 3.7), 1.5)
    assert np.max(np.abs(new[0] - e)) < 4e-16


def test_refine_zero_histogram_is_skipped():
    e = vegas.uniform_grid(2, 10)
    assert np.array_equal(vegas.refine(e, np.zeros((2, 10)), 1.5), e)


def test_refine_three_bin_worked_example():
    # d = (1, 0, 0) on a uniform 3-bin grid, alpha = 1.5.  By hand:
    # smoothed (1/2, 1/3, 0) -> p = (0.6, 0.4, 0);
    # r = (((1-.6)/ln(1/.6))^1.5, ((1-.4)/ln(1/.4))^1.5, 0)
    #   = (0.6929166164094640696, 0.5298792768219772301, 0),  R/3 = 0.40759863107714709992
    # e1 = (R/3)/r0 * 1/3 = 0.19607873031401203752
    # e2 = 1/3 + (2R/3 - r0)/r1 * 1/3 = 0.41025692146220228002
    e = vegas.uniform_grid(1, 3)
    new = vegas.refine(e, np.array([[1.0, 0.0, 0.0]]), 1.5)
    assert new[0] == pytest.approx([0.0, 0.19607873031401203752, 0.41025692146220228002, 1.0], rel=1e-14)


def test_refine_equal_mass_property():
    # The damped weights r (spread uniformly in each old bin) must give every
    # new bin the same mass R/N; check with the piecewise-linear cumulative.
    rng = np.random.default_rng(3)
    nb = 50
    e = vegas.uniform_grid(1, nb)
    hist = rng.gamma(0.5, size=(1, nb))
    new = vegas.refine(e, hist, 1.5)[0]
    d = hist[0]
    sm = np.empty(nb)
    sm[0] = (d[0] + d[1]) / 2
    sm[-1] = (d[-2] + d[-1]) / 2
    sm[1:-1] = (d[:-2] + d[1:-1] + d[2:]) / 3
    p = sm / sm.sum()
    r = np.where(p > 0, ((1 - p) / np.log(1 / p)) ** 1.5, 0.0)
    cum = np.concatenate([[0.0], np.cumsum(r)])
    C = np.interp(new, e[0], cum)
    assert np.allclose(C, np.arange(nb + 1) * r.sum() / nb, rtol=0, atol=1e-13 * r.sum())
    assert new[0] == 0.0 and new[-1] == 1.0 and np.all(np.diff(new) > 0)


def test_histogram_and_sums_match_brute_force():
    f = lambda x: gauss(x, 0.5, 0.2)
    e = vegas.uniform_grid(2, 5)
    r = vegas.iteration(f, e, seed=11, stream=0, it=0, n=2000)
    w = r["w"]
    assert r["s1"] == pytest.approx(math.fsum(w), rel=1e-16)
    _, _, idx = vegas.vegas_map(sample_uniforms(11, 0, 0, np.arange(2000, dtype=np.uint64), 2), e)
    for j in range(2):
        for i in range(5):
            assert r["hist"][j, i] == pytest.approx(sum(float(v) ** 2 for v in w[idx[:, j] == i]), rel=1e-13)
    assert r["hist"].sum(axis=1) == pytest.approx([r["s2"]] * 2, rel=1e-13)


def test_c0_estimate_consistent_with_closed_form():
    f = lambda x: gauss(x, C0["centre"], C0["sigma"])
    I = gauss_integral(4, C0["centre"], C0["sigma"])
    res = vegas.run(f, 4, C0["n_bins"], C0["alpha"], C0["iterations"], C0["n_per_iter"], C0["seed"])
    assert abs(res["mean"] - I) < 4 * res["sigma"]
    assert 0.2 < res["chi2_dof"] < 3.0
    # adaptation: the last iteration's error is far below the first one's
    assert res["iterations"][-1]["var"] < 0.05 * res["iterations"][0]["var"]


def test_pulls_over_seeds():
    """Unbiasedness and sigma-consistency of the combined estimate (VEGAS
    section, the chi^2 check of the combination): over 200 independent seeds
    the pull (E - I)/sigma has mean 0 +- 0.2 and spread 1 +- 0.15 (about 3
    standard errors each at 200 draws), and the mean chi^2/dof is near 1."""
    f = lambda x: gauss(x, 0.5, 0.15)
    I = gauss_integral(2, 0.5, 0.15)
    pulls, chi2 = [], []
    for seed in range(200):
        res = vegas.run(f, 2, 20, 1.5, 4, 4000, seed)
        pulls.append((res["mean"] - I) / res["sigma"])
        chi2.append(res["chi2_dof"])
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.2
    assert abs(pulls.std() - 1.0) < 0.15
    assert abs(np.mean(chi2) - 1.0) < 0.25


def test_converged_grid_matches_gaussian_quantiles():
    # For a separable integrand the adapted grid puts equal shares of the
    # 1-d marginal in each bin: edges approach the normal quantiles.
    c, s, nb = 0.5, 0.1, 20
    f = lambda x: gauss(x, c, s)
    res = vegas.run(f, 1, nb, 1.5, 15, 20000, seed=5)
    e = res["edges"][0]
    Z = 0.5 * (erf((1 - c) / (s * math.sqrt(2))) + erf(c / (s * math.sqrt(2))))
    lo = 0.5 * (1 + erf((0 - c) / (s * math.sqrt(2))))
    q = c + s * ndtri(lo + Z * np.arange(1, nb) / nb)
    widths = np.diff(e)
    assert np.all(np.abs(e[1:-1] - q) < 1.5 * np.maximum(widths[:-1], widths[1:]))


def test_refine_skips_non_finite_histograms():
    """A dimension whose histogram holds a non-finite weight (an iteration the
    combination excludes) keeps its edges; the other dimensions refine as
    they would alone."""
    rng = np.random.default_rng(4)
    e = vegas.uniform_grid(3, 10)
    h = rng.uniform(0.1, 2.0, size=(3, 10))
    ref = vegas.refine(e, h, 1.5)
    for bad in (np.nan, np.inf):
        hb = h.copy()
        hb[1, 4] = bad
        out = vegas.refine(e, hb, 1.5)
        assert np.array_equal(out[1], e[1])
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[2], ref[2])

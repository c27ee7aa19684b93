"""Pins of the oracle's behaviour outside the PDF grid and below the alpha_s
table (error, freeze and continuation modes)."""
import math

import numpy as np
import pytest

from oracle import pdf
from oracle import pdf_extrap as pe
from synth import synthetic_pdf_grid, synthetic_alphas, PdfGridData
from synth.alphas import AlphasTable

XK = np.geomspace(1e-6, 1.0, 20)
Q2S = [np.array([1.0, 2.0, 4.0, 8.0, 16.0]), np.geomspace(16.0, 4096.0, 6)]


def make_grid(func, n_flav=2, x_knots=XK, q2_subs=Q2S):
    xf = []
    for q2 in q2_subs:
        A = np.log(x_knots)[None, :]
        B = np.log(q2)[:, None]
        xf.append(np.stack([func(A, B) * (f + 1) for f in range(n_flav)]))
    return PdfGridData(x_knots=np.asarray(x_knots), q2_knots=[np.asarray(q) for q in q2_subs], xf=xf,
                       params={}, lambda_qcd=0.2, q0=1.0)


@pytest.fixture(scope="module")
def syn():
    return synthetic_pdf_grid()


def out_queries(grid, rng, n=40):
    """Points in every outside region (low x, high Q^2, low Q^2, corners)."""
    x0, x1 = grid.x_knots[0], grid.x_knots[-1]
    q0, q1 = grid.q2_knots[0][0], grid.q2_knots[-1][-1]
    lx_in = rng.uniform(math.log(x0), math.log(x1), n)
    lq_in = rng.uniform(math.log(q0), math.log(q1), n)
    lx_lo = math.log(x0) - rng.uniform(0.01, 8.0, n)
    lq_lo = math.log(q0) - rng.uniform(0.01, 6.0, n)
    lq_hi = math.log(q1) + rng.uniform(0.01, 6.0, n)
    xs = np.concatenate([lx_lo, lx_in, lx_in, lx_lo, lx_lo])
    qs = np.concatenate([lq_in, lq_hi, lq_lo, lq_hi, lq_lo])
    return np.exp(xs), np.exp(qs)


def test_inside_values_unchanged(syn):
    rng = np.random.default_rng(1)
    x = np.exp(rng.uniform(math.log(1e-9), 0.0, 500))
    q2 = np.exp(rng.uniform(math.log(1.0), math.log(1e10), 500))
    ref = pdf.interp(syn, x, q2)
    for mode in (pe.ERROR, pe.FREEZE, pe.CONTINUE):
        assert np.array_equal(pe.interp_extrap(syn, x, q2, mode), ref)


def test_error_mode_and_invalid_points(syn):
    rng = np.random.default_rng(2)
    x, q2 = out_queries(syn, rng)
    assert np.all(np.isnan(pe.interp_extrap(syn, x, q2, pe.ERROR)))
    bad_x = np.array([0.0, -1e-3, np.nan, 0.5, 0.5, 0.5, 1.5])
    bad_q = np.array([100.0, 100.0, 100.0, 0.0, -5.0, np.inf, 100.0])
    for mode in (pe.ERROR, pe.FREEZE, pe.CONTINUE):
        got = pe.interp_extrap(syn, bad_x, bad_q, mode)
        expect_nan = [True] * 6 + [mode != pe.FREEZE]
        assert list(np.isnan(got).all(axis=0)) == expect_nan


def test_freeze_constant_along_outward_directions(syn):
    x0, x1 = syn.x_knots[0], syn.x_knots[-1]
    q0, q1 = syn.q2_knots[0][0], syn.q2_knots[-1][-1]
    for x in (1e-4, 0.3):
        at_edge = pdf.interp(syn, x, q1)
        assert np.array_equal(pe.interp_extrap(syn, [x, x], [1.5 * q1, 1e6 * q1], pe.FREEZE),
                              np.repeat(at_edge, 2, axis=1))
        at_edge = pdf.interp(syn, x, q0)
        assert np.array_equal(pe.interp_extrap(syn, [x, x], [0.9 * q0, 1e-6 * q0], pe.FREEZE),
                              np.repeat(at_edge, 2, axis=1))
    for q2 in (3.0, 1e4):
        at_edge = pdf.interp(syn, x0, q2)
        assert np.array_equal(pe.interp_extrap(syn, [x0 / 2, 1e-30], [q2, q2], pe.FREEZE),
                              np.repeat(at_edge, 2, axis=1))
    corner = pdf.interp(syn, x0, q0)
    assert np.array_equal(pe.interp_extrap(syn, [1e-20], [1e-3 * q0], pe.FREEZE), corner)
    assert np.array_equal(pe.interp_extrap(syn, [2.0], [1e3 * q1], pe.FREEZE), pdf.interp(syn, x1, q1))


def test_low_x_power_law_continued_exactly():
    # x^-0.3 times a function linear in ln Q^2: every interpolation along
    # the x_0 and x_1 columns reproduces it, and the log branch continues the
    # power law exactly
    lam = 0.3
    g = make_grid(lambda A, B: np.exp(-lam * A) * (2.0 + 0.05 * B))
    rng = np.random.default_rng(3)
    x = np.exp(math.log(XK[0]) - rng.uniform(0.0, 20.0, 300))
    q2 = np.exp(rng.uniform(0.0, math.log(4096.0), 300))
    got = pe.interp_extrap(g, x, q2, pe.CONTINUE)
    exact = x ** -lam * (2.0 + 0.05 * np.log(q2))
    assert np.allclose(got[0], exact, rtol=1e-12, atol=0)
    assert np.allclose(got[1], 2 * exact, rtol=1e-12, atol=0)


def test_low_x_linear_branch_continued_exactly():
    # values below 1e-3 and linear in ln x: the straight line in xf continues it
    g = make_grid(lambda A, B: 4e-4 + 2e-5 * A + 0.0 * B)
    assert g.xf[0].max() <= 1e-3  # both flavours on the linear branch
    rng = np.random.default_rng(4)
    x = np.exp(math.log(XK[0]) - rng.uniform(0.0, 30.0, 200))
    q2 = np.exp(rng.uniform(0.0, math.log(4096.0), 200))
    got = pe.interp_extrap(g, x, q2, pe.CONTINUE)
    exact = 4e-4 + 2e-5 * np.log(x)
    assert np.allclose(got[0], exact, rtol=0, atol=1e-17)
    assert np.allclose(got[1], 2 * exact, rtol=0, atol=1e-17)
    assert np.any(exact < 0.0)  # the line is followed through zero


def test_high_q_power_law_continued_exactly():
    kap = 0.1
    g = make_grid(lambda A, B: (2.0 + 0.1 * A) * np.exp(kap * B))
    rng = np.random.default_rng(5)
    x = np.exp(rng.uniform(math.log(XK[0]), 0.0, 300))
    q2 = 4096.0 * np.exp(rng.uniform(0.0, 15.0, 300))
    got = pe.interp_extrap(g, x, q2, pe.CONTINUE)
    exact = (2.0 + 0.1 * np.log(x)) * q2 ** kap
    assert np.allclose(got[0], exact, rtol=1e-12, atol=0)


def test_corner_low_x_high_q_separable_power_law():
    g = make_grid(lambda A, B: np.exp(-0.25 * A + 0.08 * B))
    rng = np.random.default_rng(6)
    x = np.exp(math.log(XK[0]) - rng.uniform(0.0, 10.0, 200))
    q2 = 4096.0 * np.exp(rng.uniform(0.0, 10.0, 200))
    got = pe.interp_extrap(g, x, q2, pe.CONTINUE)
    assert np.allclose(got[0], x ** -0.25 * q2 ** 0.08, rtol=1e-12, atol=0)


def test_low_q_hand_computed_value():
    # one flavour, rows 2 (Q^2 = 1) and 3 (Q^2 = e) in every x: gamma =
    # (3 - 2)/(1 * 2) = 0.5; at Q^2 = 0.5: r = 0.5, exponent (0.5-1)*0.5+1 =
    # 0.75, xf = 2 * 2^-0.75 = 1.18920711500272106671749997056...
    xk = np.array([1e-3, 1e-2, 1e-1, 1.0])
    q2s = [np.array([1.0, math.e, math.e ** 2])]
    vals = np.array([[2.0] * 4, [3.0] * 4, [3.5] * 4])[None]
    g = PdfGridData(x_knots=xk, q2_knots=q2s, xf=[vals], params={}, lambda_qcd=0.2, q0=1.0)
    got = pe.interp_extrap(g, [0.05, 1e-5], [0.5, 0.5], pe.CONTINUE)
    assert got[0, 0] == pytest.approx(1.1892071150027210667, rel=1e-15)
    # low x at low Q^2: rows constant in x, so the x rule changes nothing
    assert got[0, 1] == pytest.approx(1.1892071150027210667, rel=1e-15)


def test_low_q_continuity_and_logarithmic_slope(syn):
    """xf and d ln xf / d ln Q^2 continuous across Q^2_min: the continuation's
    slope just below (from the extrapolated values) against the in-grid
    interpolant's slope just above (a finite difference of pdf.interp)."""
    q0 = syn.q2_knots[0][0]
    rng = np.random.default_rng(7)
    d = 1e-6
    xs = np.concatenate([np.exp(rng.uniform(math.log(1e-9), math.log(0.9), 30)), [1e-12, 1e-10]])
    checked = 0
    for x in xs:
        at = pe.interp_extrap(syn, x, q0, pe.CONTINUE)[:, 0]
        below1 = pe.interp_extrap(syn, x, q0 * math.exp(-d), pe.CONTINUE)[:, 0]
        below0 = pe.interp_extrap(syn, x, q0 * math.exp(-1e-13), pe.CONTINUE)[:, 0]
        above = pe.interp_extrap(syn, x, q0 * math.exp(d), pe.CONTINUE)[:, 0]
        nz = np.abs(at) > 1e-12
        assert np.all(below0[~nz] == 0.0) or np.allclose(below0[~nz], at[~nz], atol=1e-12)
        assert np.allclose(below0[nz], at[nz], rtol=1e-11, atol=0)
        # ln |xf|: flavours on the linear branch may have crossed zero at small x
        la, lb1, lab = np.log(np.abs(at[nz])), np.log(np.abs(below1[nz])), np.log(np.abs(above[nz]))
        slope_below = (la - lb1) / d
        slope_above = (lab - la) / d
        assert np.allclose(slope_below, slope_above, rtol=0, atol=2e-4)
        checked += nz.sum()
    assert checked > 200


def test_low_q_tends_to_linear_damping(syn):
    q0 = syn.q2_knots[0][0]
    for x in (1e-7, 1e-3, 0.2):
        g0 = pdf.interp(syn, x, q0)[:, 0]
        nz = g0 != 0.0
        for r in (1e-9, 1e-12):
            v = pe.interp_extrap(syn, x, r * q0, pe.CONTINUE)[:, 0]
            assert np.allclose(v[nz] / (g0[nz] * r), 1.0, rtol=0, atol=1e-6)
            assert np.all(v[~nz] == 0.0)


def test_low_x_continuous_at_x0_in_every_q_region(syn):
    x0 = syn.x_knots[0]
    for q2 in (0.5 * syn.q2_knots[0][0], 7.0, 1e3, 3e10):
        at = pe.interp_extrap(syn, x0, q2, pe.CONTINUE)[:, 0]
        just_below = pe.interp_extrap(syn, x0 * (1 - 1e-12), q2, pe.CONTINUE)[:, 0]
        assert np.allclose(just_below, at, rtol=1e-9, atol=1e-14)


def test_high_q_continuous_at_q2max(syn):
    q1 = syn.q2_knots[-1][-1]
    rng = np.random.default_rng(8)
    for x in np.exp(rng.uniform(math.log(1e-9), 0.0, 20)):
        at = pdf.interp(syn, x, q1)[:, 0]
        up = pe.interp_extrap(syn, x, q1 * (1 + 1e-12), pe.CONTINUE)[:, 0]
        assert np.allclose(up, at, rtol=1e-9, atol=1e-14)


def test_alphas_modes():
    tab = synthetic_alphas(synthetic_pdf_grid())
    q0, v0 = tab.q2_knots[0][0], tab.values[0][0]
    top = tab.values[-1][-1]
    q2 = np.array([0.5 * q0, 1e-3 * q0, 10 * tab.q2_knots[-1][-1], 0.0, -1.0, np.nan])
    e = pe.alphas_extrap(tab, q2, pe.ERROR)
    assert np.isnan(e[[0, 1, 3, 4, 5]]).all() and e[2] == top
    f = pe.alphas_extrap(tab, q2, pe.FREEZE)
    assert f[0] == v0 and f[1] == v0 and f[2] == top and np.isnan(f[3:]).all()
    c = pe.alphas_extrap(tab, q2, pe.CONTINUE)
    assert c[2] == top and np.isnan(c[3:]).all()
    assert c[1] > c[0] > v0  # alpha_s grows towards low scales
    # continuity at the lowest knot
    assert pe.alphas_extrap(tab, [q0 * (1 - 1e-13)], pe.CONTINUE)[0] == pytest.approx(v0, rel=1e-12)


def test_alphas_power_law_continued_exactly():
    q = [np.geomspace(1.0, 100.0, 6), np.geomspace(100.0, 1e4, 5)]
    tab = AlphasTable(q, [0.3 * qq ** -0.05 for qq in q])
    q2 = np.geomspace(1e-6, 0.99, 50)
    got = pe.alphas_extrap(tab, q2, pe.CONTINUE)
    assert np.allclose(got, 0.3 * q2 ** -0.05, rtol=1e-13, atol=0)


def test_low_x_uses_the_two_lowest_knots(syn):
    # one knot spacing below x_0 at a Q^2 knot: the line through the node
    # values F0 (x_0) and F1 (x_1) gives F0^2/F1 on the log branch, 2 F0 - F1
    # on the linear one
    xk = syn.x_knots
    x = xk[0] * xk[0] / xk[1]
    for s, j in ((1, 2), (2, 5), (2, 20)):
        q2 = syn.q2_knots[s][j]
        F0, F1 = syn.xf[s][:, j, 0], syn.xf[s][:, j, 1]
        got = pe.interp_extrap(syn, [x], [q2], pe.CONTINUE)[:, 0]
        pos = (F0 > 1e-3) & (F1 > 1e-3)
        assert pos.any() and (~pos).any()
        assert np.allclose(got[pos], F0[pos] ** 2 / F1[pos], rtol=1e-12, atol=0)
        assert np.allclose(got[~pos], 2 * F0[~pos] - F1[~pos], rtol=0, atol=1e-15)


def test_log_branch_needs_both_values_above_threshold():
    # values 2e-3 and 5e-4 at the two lowest knots (either order): the
    # straight line is drawn through xf, not ln xf
    xk = np.array([1e-4, 1e-3, 1e-2, 1e-1, 1.0])
    q2s = [np.array([1.0, 4.0, 16.0])]
    for a, b in ((2e-3, 5e-4), (5e-4, 2e-3), (2e-3, 4e-3)):
        row = np.array([a, b, 1.0, 1.0, 1.0])
        g = PdfGridData(x_knots=xk, q2_knots=q2s, xf=[np.tile(row, (1, 3, 1))], params={}, lambda_qcd=0.2, q0=1.0)
        got = pe.interp_extrap(g, [1e-5], [4.0], pe.CONTINUE)[0, 0]
        expect = a * a / b if (a > 1e-3 and b > 1e-3) else 2 * a - b
        assert got == pytest.approx(expect, rel=1e-13)

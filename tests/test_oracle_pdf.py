"""Pins of the oracle's log-bicubic PDF interpolation."""
import math

import numpy as np
import pytest
from scipy.special import betainc, beta as beta_fn

from oracle import pdf
from synth import synthetic_pdf_grid, PdfGridData, FLAVOURS
from synth.pdfgrid import momentum_sum_at_q0


def make_grid(x_knots, q2_subs, func, n_flav=2):
    xf = []
    for q2 in q2_subs:
        A = np.log(x_knots)[None, :]
        B = np.log(q2)[:, None]
        xf.append(np.stack([func(A, B) * (f + 1) for f in range(n_flav)]))
    return PdfGridData(x_knots=np.asarray(x_knots), q2_knots=[np.asarray(q) for q in q2_subs], xf=xf,
                       params={}, lambda_qcd=0.2, q0=1.0)


def test_hermite_kernel_reproduces_cubics():
    # p(t) = 1 + 2t - 3t^2 + 4t^3: p(0)=1, p(1)=4, p'(0)=2, p'(1)=8
    t = np.linspace(0, 1, 11)
    assert np.allclose(pdf.hermite(1.0, 4.0, 2.0, 8.0, t), 1 + 2 * t - 3 * t**2 + 4 * t**3, rtol=0, atol=1e-14)


def test_tensor_hermite_with_exact_derivatives_reproduces_bicubics():
    # the 2-d scheme is a tensor product of the 1-d kernel: with exact
    # derivatives it is exact for every bicubic polynomial.
    rng = np.random.default_rng(0)
    C = rng.normal(size=(4, 4))
    P = lambda s, t: sum(C[i, j] * s**i * t**j for i in range(4) for j in range(4))
    Ps = lambda s, t: sum(i * C[i, j] * s**(i - 1) * t**j for i in range(1, 4) for j in range(4))
    Pt = lambda s, t: sum(j * C[i, j] * s**i * t**(j - 1) for i in range(4) for j in range(1, 4))
    Pst = lambda s, t: sum(i * j * C[i, j] * s**(i - 1) * t**(j - 1) for i in range(1, 4) for j in range(1, 4))
    s, t = rng.uniform(size=50), rng.uniform(size=50)
    # interpolate in s at t = 0 and t = 1 for value and t-derivative, then in t
    v0 = pdf.hermite(P(0, 0), P(1, 0), Ps(0, 0), Ps(1, 0), s)
    v1 = pdf.hermite(P(0, 1), P(1, 1), Ps(0, 1), Ps(1, 1), s)
    d0 = pdf.hermite(Pt(0, 0), Pt(1, 0), Pst(0, 0), Pst(1, 0), s)
    d1 = pdf.hermite(Pt(0, 1), Pt(1, 1), Pst(0, 1), Pst(1, 1), s)
    assert np.allclose(pdf.hermite(v0, v1, d0, d1, t), P(s, t), rtol=1e-12, atol=1e-12)


def test_node_values_exact():
    g = synthetic_pdf_grid()
    for s, q2 in enumerate(g.q2_knots):
        for j in range(len(q2) - 1):  # the top knot belongs to the next subgrid
            i = np.arange(0, 195, 7)
            out = pdf.interp(g, g.x_knots[i], np.full(i.shape, q2[j]))
            ref = g.xf[s][:, j, i]
            assert np.allclose(out, ref, rtol=1e-13, atol=0)


def test_quadratics_reproduced_on_uniform_spacing():
    xk = np.exp(np.linspace(np.log(1e-4), 0.0, 30))
    q2 = [np.exp(np.linspace(np.log(2.0), np.log(1e4), 20))]
    quad = lambda A, B: 3 + 0.7 * A - 0.4 * B + 0.05 * A * A + 0.02 * A * B - 0.03 * B * B
    g = make_grid(xk, q2, quad)
    rng = np.random.default_rng(1)
    # bicubic zone: cells 1..n-3 in both axes
    a = rng.uniform(np.log(xk[1]), np.log(xk[-3]), 2000)
    b = rng.uniform(np.log(q2[0][1]), np.log(q2[0][-3]), 2000)
    out = pdf.interp(g, np.exp(a), np.exp(b))
    assert np.allclose(out[0], quad(a, b), rtol=1e-12, atol=0)
    assert np.allclose(out[1], 2 * quad(a, b), rtol=1e-12, atol=0)


def test_linear_reproduced_on_nonuniform_spacing_everywhere():
    rng = np.random.default_rng(2)
    xk = np.sort(np.exp(rng.uniform(np.log(1e-5), 0.0, 25)))
    xk[-1] = 1.0
    q2 = [np.sort(np.exp(rng.uniform(np.log(1.0), np.log(1e3), 9))),
          np.sort(np.exp(rng.uniform(np.log(1e3), np.log(1e6), 12)))]
    q2[1][0] = q2[0][-1]
    lin = lambda A, B: 1.5 - 0.3 * A + 0.2 * B
    g = make_grid(xk, q2, lin)
    a = rng.uniform(np.log(xk[0]), 0.0, 4000)
    b = rng.uniform(np.log(q2[0][0]), np.log(q2[1][-1]), 4000)
    out = pdf.interp(g, np.exp(a), np.exp(b))
    assert np.allclose(out[0], lin(a, b), rtol=1e-11, atol=1e-12)


def test_bilinear_zone_reproduces_bilinear():
    xk = np.exp(np.linspace(np.log(1e-3), 0.0, 12))
    q2 = [np.exp(np.linspace(0.0, np.log(1e3), 8))]
    bil = lambda A, B: 2 + A - 0.5 * B + 0.25 * A * B
    g = make_grid(xk, q2, bil)
    rng = np.random.default_rng(3)
    # edge cells: i = 0 and i = n_x - 2 use the bilinear rule
    for lo, hi in ((0, 1), (10, 11)):
        a = rng.uniform(np.log(xk[lo]), np.log(xk[hi]), 500)
        b = rng.uniform(0.0, np.log(1e3), 500)
        out = pdf.interp(g, np.exp(a), np.exp(b))
        assert np.allclose(out[0], bil(a, b), rtol=1e-12, atol=1e-13)


def test_c1_continuity_across_interior_knots():
    g = synthetic_pdf_grid()
    q2 = np.full(2, 1.0e3)
    for i in (20, 100, 150):
        xk = g.x_knots[i]
        h = 1e-6
        left = pdf.interp(g, np.array([xk * math.exp(-2 * h), xk * math.exp(-h)]), q2)
        right = pdf.interp(g, np.array([xk * math.exp(h), xk * math.exp(2 * h)]), q2)
        at = pdf.interp(g, np.array([xk]), q2[:1])[:, 0]
        dl = (left[:, 1] - left[:, 0]) / h
        dr = (right[:, 1] - right[:, 0]) / h
        scale = np.abs(at) + 1e-300
        assert np.all(np.abs(dl - dr) <= 1e-4 * np.maximum(np.abs(dl), scale))


def test_matches_brute_force_scalar_on_tiny_grid():
    rng = np.random.default_rng(4)
    xk = np.sort(np.exp(rng.uniform(np.log(1e-3), 0.0, 7)))
    xk[0], xk[-1] = 1e-3, 1.0
    q2 = [np.array([1.0, 2.0, 3.5]), np.array([3.5, 10.0, 40.0, 90.0, 300.0])]
    g = PdfGridData(x_knots=xk, q2_knots=q2, xf=[rng.uniform(0.1, 2.0, (2, 3, 7)), rng.uniform(0.1, 2.0, (2, 5, 7))],
                    params={}, lambda_qcd=0.2, q0=1.0)
    x = np.exp(rng.uniform(np.log(1e-3), 0.0, 300))
    q = np.exp(rng.uniform(0.0, np.log(300.0), 300))
    q = np.concatenate([q, [3.5, 1.0, 300.0]])
    x = np.concatenate([x, [0.5, 1e-3, 1.0]])
    out = pdf.interp(g, x, q)
    for k in range(len(x)):
        for f in range(2):
            assert out[f, k] == pytest.approx(pdf.interp_scalar(g, f, float(x[k]), float(q[k])), rel=1e-13, abs=1e-15)


def test_threshold_belongs_to_upper_subgrid_and_out_of_grid_is_nan():
    xk = np.array([1e-3, 1e-2, 1e-1, 1.0])
    q2 = [np.array([1.0, 2.0]), np.array([2.0, 4.0])]
    g = PdfGridData(x_knots=xk, q2_knots=q2, xf=[np.ones((1, 2, 4)), 2 * np.ones((1, 2, 4))],
                    params={}, lambda_qcd=0.2, q0=1.0)
    out = pdf.interp(g, np.array([0.05, 0.05, 0.05, 0.05, 1e-4, 1.5]), np.array([1.5, 2.0, 4.0, 5.0, 1.5, 1.5]))
    assert list(out[0, :3]) == [1.0, 2.0, 2.0]
    assert np.all(np.isnan(out[0, 3:]))


def _simpson_lnx(g, q2, k_lo, k_hi, sub=20):
    """int xf dx over [x_klo, x_khi] of the interpolated grid (Simpson in ln x)."""
    lx = np.log(g.x_knots)
    total = 0.0
    for k in range(k_lo, k_hi):
        t = np.linspace(lx[k], lx[k + 1], sub + 1)
        x = np.exp(t)
        if k + 1 == len(lx) - 1:
            x[-1] = 1.0
        v = pdf.interp(g, x, np.full(x.shape, q2)).sum(axis=0) * x  # xf dx = xf x d(ln x)
        h = (t[-1] - t[0]) / sub
        total += h / 3 * (v[0] + v[-1] + 4 * v[1:-1:2].sum() + 2 * v[2:-1:2].sum())
    return total


def _exact_momentum(g, x_lo, x_hi):
    """int_{x_lo}^{x_hi} sum_f xf dx of the continuous functions at Q0."""
    tot = 0.0
    for pid in FLAVOURS:
        if abs(pid) in (4, 5):
            continue
        A0, a0, b0, c = g.params[pid]
        for aa, cc in ((a0 + 1.0, 1.0), (a0 + 1.5, c)):
            B = beta_fn(aa, b0 + 1.0)
            tot += A0 * cc * B * (betainc(aa, b0 + 1.0, x_hi) - betainc(aa, b0 + 1.0, x_lo))
    return tot


def test_synthetic_grid_momentum_sum_rule():
    # The continuous functions satisfy sum_f int_0^1 xf dx = 1 at Q0 exactly
    # (Beta-function normalisation).  The interpolated grid must reproduce the
    # momentum integral for x <= 0.35 to the interpolation error (cells of
    # width 0.106 in ln x; measured ~1e-4 relative), and over the whole range
    # up to the error of the last, bilinear cell [0.9, 1], where (1-x)^b is
    # poorly resolved by log-spaced knots (~1e-3).  A dropped flavour, term or
    # subgrid would show up as an O(1e-2) or larger deviation.
    g = synthetic_pdf_grid()
    assert momentum_sum_at_q0(g) == pytest.approx(1.0, rel=1e-14)
    q0sq = g.q2_knots[0][0]
    xk = g.x_knots
    inner = _simpson_lnx(g, q0sq, 1, 185)
    assert inner == pytest.approx(_exact_momentum(g, xk[1], xk[185]), rel=2e-4)
    full = _simpson_lnx(g, q0sq, 0, len(xk) - 1) + _exact_momentum(g, 0.0, xk[0])
    assert full == pytest.approx(1.0, abs=1.5e-3)

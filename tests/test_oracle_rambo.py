"""Pins of the oracle's RAMBO generator and unweighting."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import rambo as orb
from oracle.philox import sample_uniforms


def lam(a, b, c):
    return a * a + b * b + c * c - 2 * a * b - 2 * a * c - 2 * b * c


def test_conservation_and_mass_shells():
    for masses, rs in (([0.0] * 2, 100.0), ([0.0] * 5, 250.0), ([173.0, 173.0], 800.0),
                       ([80.4, 4.7, 0.0, 91.2], 500.0), ([1.0] * 8, 20.0)):
        k, w = orb.generate(5, 1, 0, 0, 2000, masses, rs)
        tot = k.sum(axis=1)
        assert np.allclose(tot[:, 0], rs, rtol=1e-13, atol=0)
        assert np.allclose(tot[:, 1:], 0.0, rtol=0, atol=1e-12 * rs)
        m2 = k[:, :, 0] ** 2 - (k[:, :, 1:] ** 2).sum(axis=2)
        assert np.allclose(m2, np.asarray(masses)[None, :] ** 2, rtol=0, atol=1e-10 * rs * rs)
        assert np.all(k[:, :, 0] > 0.0) and np.all(np.isfinite(w)) and np.all(w > 0.0)


def test_massless_volumes_closed_forms():
    # two-body 1/(8 pi); three-body s/(256 pi^3)
    assert orb.massless_weight(2, 123.0) == pytest.approx(1.0 / (8 * math.pi), rel=1e-15)
    assert orb.massless_weight(3, 91.0) == pytest.approx(91.0 ** 2 / (256 * math.pi ** 3), rel=1e-14)
    _, w = orb.generate(1, 0, 0, 0, 10, [0.0, 0.0, 0.0], 91.0)
    assert np.all(w == orb.massless_weight(3, 91.0))


def test_massive_two_body_weight_is_beta_over_8pi_event_by_event():
    # 1e-9: the boost x H_b cancels when the q's are nearly collinear (M small,
    # gamma large) and the massless energies then carry rounding of order
    # gamma^2 ulp; unequal masses feel it through xi
    for m1, m2, rs in ((173.0, 173.0, 400.0), (80.4, 4.7, 120.0), (0.0, 173.0, 300.0)):
        _, w = orb.generate(9, 2, 1, 7, 20_000, [m1, m2], rs)
        beta = math.sqrt(lam(rs * rs, m1 * m1, m2 * m2)) / (rs * rs)
        assert np.allclose(w, beta / (8 * math.pi), rtol=1e-9, atol=0)


def dalitz_volume(rs, m1, m2, m3):
    """Three-body phase-space volume from the Dalitz plot: (1/(128 pi^3 s))
    times the area in (m12^2, m23^2)."""
    s = rs * rs

    def width(m12sq):
        m12 = math.sqrt(m12sq)
        e2 = (m12sq - m1 * m1 + m2 * m2) / (2 * m12)
        e3 = (s - m12sq - m3 * m3) / (2 * m12)
        p2 = math.sqrt(max(e2 * e2 - m2 * m2, 0.0))
        p3 = math.sqrt(max(e3 * e3 - m3 * m3, 0.0))
        return (e2 + e3) ** 2 - (p2 - p3) ** 2 - ((e2 + e3) ** 2 - (p2 + p3) ** 2)

    area, _ = integrate.quad(width, (m1 + m2) ** 2, (rs - m3) ** 2, epsabs=0, epsrel=1e-12, limit=200)
    return area / (128 * math.pi ** 3 * s)


def test_massive_three_body_volume_against_dalitz_quadrature():
    assert dalitz_volume(91.0, 0, 0, 0) == pytest.approx(91.0 ** 2 / (256 * math.pi ** 3), rel=1e-10)
    rs, masses = 300.0, [80.4, 91.2, 4.7]
    ref = dalitz_volume(rs, *masses)
    _, w = orb.generate(3, 4, 0, 0, 400_000, masses, rs)
    mean, err = w.mean(), w.std() / math.sqrt(w.size)
    assert abs(mean - ref) < 4 * err
    assert err / ref < 3e-3  # the test resolves a wrong weight factor


def test_massless_three_body_points_flat_in_the_dalitz_plot():
    # flat phase space: (m12^2, m23^2, m13^2)/s is uniform on the simplex,
    # so E[(m12^2/s)^2] = 1/6 and E[(m12^2/s)(m23^2/s)] = 1/12
    rs = 50.0
    k, _ = orb.generate(11, 0, 0, 0, 200_000, [0.0, 0.0, 0.0], rs)

    def inv(a, b):
        v = k[:, a] + k[:, b]
        return (v[:, 0] ** 2 - (v[:, 1:] ** 2).sum(axis=1)) / rs ** 2

    x, y = inv(0, 1), inv(1, 2)
    for vals, expect in ((x * x, 1 / 6), (x * y, 1 / 12), (x, 1 / 3)):
        assert abs(vals.mean() - expect) < 4 * vals.std() / math.sqrt(vals.size)


def test_isotropy():
    k, _ = orb.generate(2, 3, 0, 0, 100_000, [0.0, 0.0], 10.0)
    for j in (1, 2, 3):
        c = k[:, 0, j] / k[:, 0, 0]
        assert abs(c.mean()) < 4 * c.std() / math.sqrt(c.size)
        assert abs((c * c).mean() - 1 / 3) < 4 * (c * c).std() / math.sqrt(c.size)


def test_xi_solution():
    k, _ = orb.generate(8, 0, 0, 0, 500, [5.0, 20.0, 0.5], 40.0)
    assert np.allclose(k[:, :, 0].sum(axis=1), 40.0, rtol=1e-15, atol=0)


def test_unweighting_rates_and_distribution():
    n = 200_000
    # equal weights: every event kept (r < 1)
    idx, wm = orb.unweight(np.full(n, 2.5), 3, 7, 0)
    assert idx.size == n and wm == 2.5
    # an all-zero sample keeps nothing (w_max = 0)
    idx0, wm0 = orb.unweight(np.zeros(10), 3, 7, 0)
    assert idx0.size == 0 and wm0 == 0.0
    # zero weights never kept, negative and NaN weights never kept
    w = np.array([0.0, -1.0, np.nan, 1.0])
    assert list(orb.unweight(w, 3, 7, 0)[0]) == [3]
    # weights x on uniform x: efficiency mean(w)/w_max = 1/2, and the kept
    # x follow the density 2x (mean 2/3)
    x = sample_uniforms(1, 2, 0, np.arange(n, dtype=np.uint64), 1)[:, 0]
    idx, wm = orb.unweight(x, 3, 7, 0)
    eff = idx.size / n
    assert abs(eff - 0.5) < 4 * math.sqrt(0.25 / n)
    kept = x[idx]
    assert abs(kept.mean() - 2 / 3) < 4 * kept.std() / math.sqrt(kept.size)
    assert np.all(np.diff(idx) > 0)
    # a given bound above the maximum lowers the efficiency in proportion
    idx2, wm2 = orb.unweight(x, 3, 7, 0, w_max=2.0 * wm)
    assert wm2 == 2.0 * wm and abs(idx2.size / n - 0.25) < 4 * math.sqrt(0.1875 / n)

"""Pins of the oracle's LO t tbar integrand."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import ttbar, vegas
from synth import C2, synthetic_pdf_grid

MT, AS = C2["m_top"], C2["alpha_s"]
G4 = (4 * math.pi * AS) ** 2


def _dsig_dcos(shat, cos, which):
    rho = 4 * MT * MT / shat
    beta = math.sqrt(1 - rho)
    t1, t2 = 0.5 * (1 - beta * cos), 0.5 * (1 + beta * cos)
    m2 = ttbar.m2_gg(t1, t2, rho, G4) if which == "gg" else ttbar.m2_qq(t1, t2, rho, G4)
    return m2 * beta / (32 * math.pi * shat)


@pytest.mark.parametrize("rs", [400.0, 600.0, 2000.0])
def test_partonic_cross_sections_closed_forms(rs):
    shat = rs * rs
    for which, closed in (("gg", ttbar.sigma_hat_gg), ("qq", ttbar.sigma_hat_qq)):
        num, _ = quad(lambda c: _dsig_dcos(shat, c, which), -1, 1, epsabs=0, epsrel=1e-13, limit=200)
        assert num == pytest.approx(closed(shat, MT, AS), rel=1e-12)


def _mandelstam_gg(s, t, u, m):
    # g g -> Q Qbar, d sigma/dt in the Mandelstam form (Combridge 1979), so
    # sum|M|^2 = 16 pi s^2 d sigma/dt.
    m2 = m * m
    a, b = m2 - t, m2 - u
    br = (6 * a * b / s**2 - m2 * (s - 4 * m2) / (3 * a * b)
          + 4.0 / 3 * (a * b - 2 * m2 * (m2 + t)) / a**2
          + 4.0 / 3 * (a * b - 2 * m2 * (m2 + u)) / b**2
          - 3 * (a * b + m2 * (u - t)) / (s * a)
          - 3 * (a * b + m2 * (t - u)) / (s * b))
    return 16 * math.pi * s * s * math.pi * AS**2 / (8 * s * s) * br


def _mandelstam_qq(s, t, u, m):
    m2 = m * m
    return 16 * math.pi * s * s * 4 * math.pi * AS**2 / (9 * s**4) * ((m2 - t)**2 + (m2 - u)**2 + 2 * m2 * s)


@pytest.mark.parametrize("rs,cos", [(360.0, 0.3), (500.0, -0.9), (1500.0, 0.99), (5000.0, 0.0)])
def test_matrix_elements_match_mandelstam_forms(rs, cos):
    s = rs * rs
    rho = 4 * MT * MT / s
    beta = math.sqrt(1 - rho)
    t1, t2 = 0.5 * (1 - beta * cos), 0.5 * (1 + beta * cos)
    t = MT * MT - s * t1
    u = MT * MT - s * t2
    assert ttbar.m2_gg(t1, t2, rho, G4) == pytest.approx(_mandelstam_gg(s, t, u, MT), rel=1e-12)
    assert ttbar.m2_qq(t1, t2, rho, G4) == pytest.approx(_mandelstam_qq(s, t, u, MT), rel=1e-12)


def _lumi_sigma(grid, tau, y):
    """(1/tau) sum_ab xf_a xf_b sigma_hat_ab(tau s) in pb, from closed forms."""
    s = C2["sqrt_s"] ** 2
    x1, x2 = math.sqrt(tau) * math.exp(y), math.sqrt(tau) * math.exp(-y)
    from oracle.pdf import interp
    f = interp(grid, np.array([x1, x2]), np.full(2, MT * MT))
    I = ttbar.IDX
    gg = f[I[21], 0] * f[I[21], 1]
    qq = sum(f[I[q], 0] * f[I[-q], 1] + f[I[-q], 0] * f[I[q], 1] for q in (1, 2, 3, 4, 5))
    sh = tau * s
    return (gg * ttbar.sigma_hat_gg(sh, MT, AS) + qq * ttbar.sigma_hat_qq(sh, MT, AS)) / tau * C2["gev2_to_pb"]


def test_angular_integral_of_integrand_gives_closed_forms():
    grid = synthetic_pdf_grid()
    rng = np.random.default_rng(0)
    xg, wg = np.polynomial.legendre.leggauss(200)
    for u1, u2 in rng.uniform(0.05, 0.95, (5, 2)):
        u3 = 0.5 * (xg + 1)
        u = np.column_stack([np.full(200, u1), np.full(200, u2), u3])
        F = ttbar.integrand(u, grid, C2["sqrt_s"], MT, AS, C2["gev2_to_pb"])
        num = 0.5 * np.sum(wg * F)
        k = ttbar.phase_space(u[:1], C2["sqrt_s"], MT)
        jac_tau_y = k["jac"][0] / 2.0  # remove J_cos = 2 (integrated here over u3)
        ref = jac_tau_y * _lumi_sigma(grid, k["tau"][0], k["y"][0])
        assert num == pytest.approx(ref, rel=1e-10)


def test_hadronic_cross_section_vegas_vs_quadrature():
    grid = synthetic_pdf_grid()
    # 2-d Gauss-Legendre over (u1, u2) of the closed-form partonic cross sections
    n = 120
    xg, wg = np.polynomial.legendre.leggauss(n)
    uu = 0.5 * (xg + 1)
    ww = 0.5 * wg
    s = C2["sqrt_s"] ** 2
    tau0 = 4 * MT * MT / s
    total = 0.0
    for u1, w1 in zip(uu, ww):
        tau = tau0 ** (1 - u1)
        jt = tau * math.log(1 / tau0)
        ly = math.log(1 / tau)
        for u2, w2 in zip(uu, ww):
            y = (u2 - 0.5) * ly
            total += w1 * w2 * jt * ly * _lumi_sigma(grid, tau, y)
    f = lambda u: ttbar.integrand(u, grid, C2["sqrt_s"], MT, AS, C2["gev2_to_pb"])
    res = vegas.run(f, 3, 50, 1.5, 5, 40000, seed=C2["seed"])
    assert abs(res["mean"] - total) < 4 * res["sigma"]
    assert res["sigma"] / res["mean"] < 5e-3
    # LO t tbar at 13 TeV is O(500 pb); the synthetic PDFs land in the same range
    assert 50.0 < total < 5000.0


def dynamic_scale_quadrature(grid, table):
    """2-d quadrature of the closed-form partonic cross sections, each with
    alpha_s and the PDFs at its own scale mu^2 = s_hat/4 (pb)."""
    from oracle.alphas import interp as alphas_interp
    from oracle.pdf import interp
    s = C2["sqrt_s"] ** 2
    tau0 = 4 * MT * MT / s
    n = 100
    xg, wg = np.polynomial.legendre.leggauss(n)
    uu, ww = 0.5 * (xg + 1), 0.5 * wg
    total = 0.0
    I = ttbar.IDX
    for u1, w1 in zip(uu, ww):
        tau = tau0 ** (1 - u1)
        sh = tau * s
        a_s = alphas_interp(table, [sh / 4])[0]
        jt = tau * math.log(1 / tau0)
        ly = math.log(1 / tau)
        ys = (uu - 0.5) * ly
        x1, x2 = math.sqrt(tau) * np.exp(ys), math.sqrt(tau) * np.exp(-ys)
        f1 = interp(grid, x1, np.full(n, sh / 4))
        f2 = interp(grid, x2, np.full(n, sh / 4))
        gg = f1[I[21]] * f2[I[21]]
        qq = sum(f1[I[q]] * f2[I[-q]] + f1[I[-q]] * f2[I[q]] for q in (1, 2, 3, 4, 5))
        lum = (gg * ttbar.sigma_hat_gg(sh, MT, a_s) + qq * ttbar.sigma_hat_qq(sh, MT, a_s)) / tau
        total += w1 * jt * ly * np.sum(ww * lum) * C2["gev2_to_pb"]
    return total


def test_dynamic_scale_hadronic_cross_section_vs_quadrature():
    """mu^2 = s_hat/4 per event with running alpha_s: VEGAS on the oracle
    integrand against 2-d quadrature of the closed-form partonic cross
    sections, each evaluated with alpha_s and the PDFs at its own scale."""
    from synth import synthetic_alphas
    grid = synthetic_pdf_grid()
    table = synthetic_alphas(grid)
    total = dynamic_scale_quadrature(grid, table)
    f = lambda u: ttbar.integrand_dynamic(u, grid, table, C2["sqrt_s"], MT, C2["gev2_to_pb"])
    res = vegas.run(f, 3, 50, 1.5, 5, 40000, seed=C2["seed"])
    assert abs(res["mean"] - total) < 4 * res["sigma"]
    assert res["sigma"] / res["mean"] < 5e-3
    # alpha_s(mu) <= alpha_s(m_t) ~ 0.108 < 0.118 for mu = sqrt(s_hat)/2 >= m_t: below the fixed-scale value
    fixed = ttbar.integrand(np.random.default_rng(0).uniform(size=(2000, 3)), grid, C2["sqrt_s"], MT, AS,
                            C2["gev2_to_pb"]).mean()
    assert total < fixed

"""LO pp -> t tbar integrand over 2 -> 2 phase space (oracle) — test infrastructure.

The thesis gives the master formula (sigma = sum_ab int dPhi_n L(x1,x2)|M|^2,
MadFlow chapter), the parton-level factorisation (PDF chapter), the two
sub-processes u ubar -> t tbar and g g -> t tbar (pp -> t tbar example) and
the two-body phase space dPhi_2 = lambda^{1/2}/(8 (2 pi)^2 M^2) dOmega
(phase-space section).  It does not print the matrix elements or a
parametrisation; the readings used here are:

  * spin- and colour-averaged LO matrix elements (Combridge 1979; Ellis,
    Stirling, Webber, "QCD and collider physics", Ch. 10), with
    tau_{1,2} = (1 -/+ beta cos theta)/2, rho = 4 m^2/s_hat, g^4 = (4 pi alpha_s)^2:
      |M|^2_qq = g^4 (4/9) (tau1^2 + tau2^2 + rho/2)
      |M|^2_gg = g^4 (1/(6 tau1 tau2) - 3/8) (tau1^2 + tau2^2 + rho - rho^2/(4 tau1 tau2))
  * 2 -> 2 phase space integrated over azimuth: dPhi_2 = beta/(16 pi) dcos,
    flux 1/(2 s_hat), so dsigma_hat/dcos = |M|^2 beta/(32 pi s_hat);
  * variables u in [0,1)^3 -> (tau, y, cos theta):
      tau = tau0^(1-u1), J_tau = tau ln(1/tau0), tau0 = 4 m^2 / s,
      y = (u2 - 1/2) ln(1/tau), J_y = ln(1/tau),
      cos = 2 u3 - 1, J_c = 2,
      x1 = sqrt(tau) e^y, x2 = sqrt(tau) e^-y, s_hat = tau s;
    dx1 dx2 = dtau dy, and f(x) = xf(x)/x gives the 1/tau factor;
  * F(u) = J_tau J_y J_c / tau * [ xg(x1) xg(x2) |M|^2_gg
        + sum_{q=d,u,s,c,b} (xq(x1) xqbar(x2) + xqbar(x1) xq(x2)) |M|^2_qq ]
        * beta / (32 pi s_hat) * 0.3893793721e9 pb GeV^2,
    PDFs at mu^2 = m_t^2, fixed alpha_s, no cuts.

Dynamic scale (the thesis's PDF tools evaluate xf at any (x, Q^2) and
alpha_s(Q) by log-cubic interpolation):
integrand_dynamic() sets mu^2 = s_hat/4 per event, with alpha_s(mu) from the
PDF set's alpha_s table.

Pins: tests/test_oracle_ttbar.py -- the partonic cross sections against
their closed forms
  sigma_qq = 8 pi alpha_s^2/(27 s_hat) beta (1 + rho/2),
  sigma_gg = pi alpha_s^2/(3 s_hat) [(1 + rho + rho^2/16) ln((1+beta)/(1-beta))
             - beta (7/4 + 31 rho/16)],
a second, independently written form of |M|^2_gg in Mandelstam variables,
and the hadronic integral against adaptive quadrature of the closed forms.
"""
import math

import numpy as np

from . import pdf as pdf_oracle

# index of each flavour in the PDF arrays (order -5..-1, g, 1..5)
IDX = {-5: 0, -4: 1, -3: 2, -2: 3, -1: 4, 21: 5, 1: 6, 2: 7, 3: 8, 4: 9, 5: 10}


def m2_qq(tau1, tau2, rho, g4):
    return g4 * (4.0 / 9.0) * (tau1 * tau1 + tau2 * tau2 + 0.5 * rho)


def m2_gg(tau1, tau2, rho, g4):
    t12 = tau1 * tau2
    return g4 * (1.0 / (6.0 * t12) - 0.375) * (tau1 * tau1 + tau2 * tau2 + rho - rho * rho / (4.0 * t12))


def sigma_hat_qq(shat, mt, alpha_s):
    rho = 4.0 * mt * mt / shat
    beta = math.sqrt(1.0 - rho)
    return 8.0 * math.pi * alpha_s ** 2 / (27.0 * shat) * beta * (1.0 + 0.5 * rho)


def sigma_hat_gg(shat, mt, alpha_s):
    rho = 4.0 * mt * mt / shat
    beta = math.sqrt(1.0 - rho)
    return math.pi * alpha_s ** 2 / (3.0 * shat) * (
        (1.0 + rho + rho * rho / 16.0) * math.log((1.0 + beta) / (1.0 - beta)) - beta * (1.75 + 31.0 * rho / 16.0))


def phase_space(u, sqrt_s, mt):
    """(tau, y, cos) map of u (n, 3).  Returns a dict of kinematics."""
    u = np.asarray(u, dtype=np.float64)
    s = sqrt_s * sqrt_s
    tau0 = 4.0 * mt * mt / s
    l0 = math.log(1.0 / tau0)
    tau = tau0 ** (1.0 - u[:, 0])
    jac_tau = tau * l0
    ltau = np.log(1.0 / tau)
    y = (u[:, 1] - 0.5) * ltau
    jac_y = ltau
    cos = 2.0 * u[:, 2] - 1.0
    jac = jac_tau * jac_y * 2.0
    sq = np.sqrt(tau)
    x1 = sq * np.exp(y)
    x2 = sq * np.exp(-y)
    shat = tau * s
    rho = 4.0 * mt * mt / shat
    beta = np.sqrt(1.0 - rho)
    tau1 = 0.5 * (1.0 - beta * cos)
    tau2 = 0.5 * (1.0 + beta * cos)
    return dict(tau=tau, y=y, cos=cos, jac=jac, x1=x1, x2=x2, shat=shat, rho=rho,
                beta=beta, tau1=tau1, tau2=tau2)


def integrand_dynamic(u, grid, alphas_table, sqrt_s, mt, gev2_to_pb):
    """F(u) in pb with the scale set per event, mu^2 = s_hat/4 (the PDFs at
    (x, mu^2) and alpha_s(mu) from the alpha_s table by the log-cubic rule);
    otherwise as integrand()."""
    from . import alphas as alphas_oracle
    k = phase_space(u, sqrt_s, mt)
    mu2 = k["shat"] / 4.0
    f1 = pdf_oracle.interp(grid, k["x1"], mu2)
    f2 = pdf_oracle.interp(grid, k["x2"], mu2)
    a_s = alphas_oracle.interp(alphas_table, mu2)
    g4 = (4.0 * math.pi * a_s) ** 2
    mgg = m2_gg(k["tau1"], k["tau2"], k["rho"], g4)
    mqq = m2_qq(k["tau1"], k["tau2"], k["rho"], g4)
    lum_gg = f1[IDX[21]] * f2[IDX[21]]
    lum_qq = np.zeros_like(lum_gg)
    for q in (1, 2, 3, 4, 5):
        lum_qq = lum_qq + f1[IDX[q]] * f2[IDX[-q]] + f1[IDX[-q]] * f2[IDX[q]]
    dps = k["beta"] / (32.0 * math.pi * k["shat"])
    return k["jac"] / k["tau"] * (lum_gg * mgg + lum_qq * mqq) * dps * gev2_to_pb


def integrand(u, grid, sqrt_s, mt, alpha_s, gev2_to_pb):
    """F(u) in pb for u (n, 3)."""
    k = phase_space(u, sqrt_s, mt)
    mu2 = mt * mt
    q2 = np.full(k["x1"].shape, mu2)
    f1 = pdf_oracle.interp(grid, k["x1"], q2)
    f2 = pdf_oracle.interp(grid, k["x2"], q2)
    g4 = (4.0 * math.pi * alpha_s) ** 2
    mgg = m2_gg(k["tau1"], k["tau2"], k["rho"], g4)
    mqq = m2_qq(k["tau1"], k["tau2"], k["rho"], g4)
    lum_gg = f1[IDX[21]] * f2[IDX[21]]
    lum_qq = np.zeros_like(lum_gg)
    for q in (1, 2, 3, 4, 5):
        lum_qq = lum_qq + f1[IDX[q]] * f2[IDX[-q]] + f1[IDX[-q]] * f2[IDX[q]]
    dps = k["beta"] / (32.0 * math.pi * k["shat"])
    return k["jac"] / k["tau"] * (lum_gg * mgg + lum_qq * mqq) * dps * gev2_to_pb

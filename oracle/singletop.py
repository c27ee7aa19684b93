"""LO s-channel single top, u dbar (c sbar) -> W* -> t bbar (oracle) — test infrastructure.

Only tests/, the smoke check and the CPU baseline of the benchmark use this
module; the library never does.

The thesis's LO example (physics-examples section): pp -> t + 1 jet with
q qbar -> t bbar as the only diagram, m_t = 173.2 GeV at the LHC Run 1
energy (the text's "8 GeV" read as 8 TeV), the cross section an integral
of |M|^2 times the luminosity over the phase space (master formula, MadFlow
chapter).  It prints no matrix element; readings used here:

  * W vertex (g/sqrt 2) gamma^mu P_L, g^2 = 4 pi alpha / s_W^2, diagonal
    CKM matrix (V_ud = V_cs = V_tb = 1), W propagator
    1/(s_hat - M_W^2 + i M_W Gamma_W), massless light quarks and b;
  * spin- and colour-averaged (colour factor 1: singlet exchange between two
    colour-singlet currents) |M|^2 = (g^4/4) |P|^2 u_hat (u_hat - m_t^2),
    u_hat = (p_q - p_bbar)^2 = -(s_hat - m_t^2)(1 + cos)/2, cos the angle
    between the quark and the top in the partonic rest frame;
  * two-body phase space with one massive particle: dPhi_2 = beta/(16 pi) dcos
    after the azimuth, beta = 1 - m_t^2/s_hat, flux 1/(2 s_hat):
    dsigma_hat/dcos = |M|^2 beta / (32 pi s_hat);
  * variables u in [0,1)^3 -> (tau, y, cos theta*) from threshold:
      tau = tau0^(1-u1), tau0 = m_t^2/s, J_tau = tau ln(1/tau0),
      y = (u2 - 1/2) ln(1/tau), J_y = ln(1/tau), cos = 2 u3 - 1, J_c = 2;
  * F(u) = J_tau J_y J_c / tau * sum_{(q,q')=(u,dbar),(c,sbar)} [xq(x1) xq'(x2)
        dsigma(cos) + xq'(x1) xq(x2) dsigma(-cos)] * 0.3893793721e9 pb GeV^2,
    PDFs at mu^2 = m_t^2, top only (no t-bar channel), no cuts.

Pins: tests/test_oracle_singletop.py -- |M|^2 against a brute-force Dirac
trace with a massive top at random momenta, sigma_hat against the textbook
pi alpha^2/(24 s_W^4) (s_hat - m_t^2)^2 (2 s_hat + m_t^2) / (s_hat^2 |s_hat -
M_W^2 + i M_W Gamma_W|^2), the beam assignment per event, and the hadronic
integral against quadrature.
"""
import math

import numpy as np

from . import pdf as pdf_oracle
from .ttbar import IDX

# (quark, antiquark) pairs that make a W+ with a diagonal CKM matrix
PAIRS = ((2, -1), (4, -3))


def m2bar(cos, shat, mt, mw, gw, sw2, alpha):
    """Spin- and colour-averaged |M|^2 of q qbar' -> t bbar."""
    g4 = (4.0 * math.pi * alpha / sw2) ** 2
    shat = np.asarray(shat, dtype=np.float64)
    uhat = -(shat - mt * mt) * (1.0 + np.asarray(cos, dtype=np.float64)) / 2.0
    p2 = 1.0 / ((shat - mw * mw) ** 2 + (mw * gw) ** 2)
    return g4 / 4.0 * p2 * uhat * (uhat - mt * mt)


def dsigma_dcos(cos, shat, mt, mw, gw, sw2, alpha):
    beta = 1.0 - mt * mt / np.asarray(shat, dtype=np.float64)
    return m2bar(cos, shat, mt, mw, gw, sw2, alpha) * beta / (32.0 * math.pi * shat)


def phase_space(u, sqrt_s, mt):
    u = np.asarray(u, dtype=np.float64)
    s = sqrt_s * sqrt_s
    tau0 = mt * mt / s
    l0 = math.log(1.0 / tau0)
    tau = tau0 ** (1.0 - u[:, 0])
    ltau = np.log(1.0 / tau)
    y = (u[:, 1] - 0.5) * ltau
    cos = 2.0 * u[:, 2] - 1.0
    jac = (tau * l0) * ltau * 2.0
    sq = np.sqrt(tau)
    return dict(tau=tau, y=y, cos=cos, jac=jac, x1=sq * np.exp(y), x2=sq * np.exp(-y), shat=tau * s)


def integrand(u, grid, sqrt_s, mt, mw, gw, sw2, alpha, gev2_to_pb):
    """F(u) in pb for u (n, 3)."""
    k = phase_space(u, sqrt_s, mt)
    q2 = np.full(k["x1"].shape, mt * mt)
    f1 = pdf_oracle.interp(grid, k["x1"], q2)
    f2 = pdf_oracle.interp(grid, k["x2"], q2)
    fwd = dsigma_dcos(k["cos"], k["shat"], mt, mw, gw, sw2, alpha)
    bwd = dsigma_dcos(-k["cos"], k["shat"], mt, mw, gw, sw2, alpha)
    tot = np.zeros_like(k["tau"])
    for q, qb in PAIRS:
        tot = tot + f1[IDX[q]] * f2[IDX[qb]] * fwd + f1[IDX[qb]] * f2[IDX[q]] * bwd
    return k["jac"] / k["tau"] * tot * gev2_to_pb


def integrand_from_config(u, grid, c):
    return integrand(u, grid, c["sqrt_s"], c["m_top"], c["m_w"], c["gamma_w"], c["sw2"], c["alpha_em"],
                     c["gev2_to_pb"])

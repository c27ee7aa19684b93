"""LO pp -> gamma*/Z -> l+ l- (Drell-Yan) integrand (oracle) — test infrastructure.

Only tests/, the smoke check and the CPU baseline of the benchmark use this
module; the library never does.

The thesis gives the master formula (sigma = sum_ab int dPhi_n L(x1,x2)|M|^2,
MadFlow chapter), the parton-level factorisation (PDF chapter) and the
two-body phase space (phase-space section); it names Drell-Yan among the
processes its tools target but prints no matrix element.  Readings used
here (standard electroweak theory, massless fermions):

  * chiral Z couplings g_L = T3 - Q s_W^2, g_R = -Q s_W^2, the Z vertex
    (e/(s_W c_W)) gamma^mu (g_L P_L + g_R P_R), the photon vertex e Q gamma^mu;
  * for q(p1) qbar(p2) -> l-(p3) l+(p4) with theta the angle between the
    quark and the l-, the helicity amplitudes (quark helicity i, lepton
    helicity j) have |A_ij|^2 = e^4 (1 + cos)^2 |F_ij|^2 for i = j and
    e^4 (1 - cos)^2 |F_ij|^2 for i != j, with
      F_ij = Q_q Q_l + g_i^q g_j^l chi,  chi = s_hat / (s_W^2 c_W^2 (s_hat - M_Z^2 + i M_Z Gamma_Z));
  * spin average 1/4 and colour average 1/N_c = 1/3:
      |M|^2 = (e^4/12) sum_ij |A_ij|^2 / e^4,  dsigma_hat/dcos = |M|^2 / (32 pi s_hat);
  * variables u in [0,1)^3 -> (tau, y, cos theta*) over the mass window
    m_lo < m_ll < m_hi:
      tau = tau_lo (tau_hi/tau_lo)^u1, J_tau = tau ln(tau_hi/tau_lo),
      y = (u2 - 1/2) ln(1/tau), J_y = ln(1/tau), cos = 2 u3 - 1, J_c = 2,
      x1 = sqrt(tau) e^y, x2 = sqrt(tau) e^-y, s_hat = tau s;
  * F(u) = J_tau J_y J_c / tau * sum_{q=d,u,s,c,b} [xq(x1) xqbar(x2) dsigma_q(cos)
        + xqbar(x1) xq(x2) dsigma_q(-cos)] * 0.3893793721e9 pb GeV^2,
    (a quark from the second beam sees the l- at pi - theta), PDFs at
    mu^2 = M_Z^2, fixed alpha, no lepton cuts beyond the mass window.

Pins: tests/test_oracle_drellyan.py -- |M|^2 against a brute-force Dirac
trace of the gamma + Z amplitudes at random momenta; the photon-only limit
against sigma_hat = 4 pi alpha^2 Q_q^2 / (9 s_hat); the Z pole, where the
interference vanishes, against sigma_gamma + 12 pi Gamma_qq Gamma_ll /
(9 M_Z^2 Gamma_Z^2) with Gamma_ff = N_c alpha M_Z (g_L^2 + g_R^2) /
(6 s_W^2 c_W^2); and the hadronic integral against quadrature.
"""
import math

import numpy as np

from . import pdf as pdf_oracle
from .ttbar import IDX

# (electric charge, weak isospin) of the up- and down-type quarks and the l-
CHARGES = {"u": (2.0 / 3.0, 0.5), "d": (-1.0 / 3.0, -0.5), "l": (-1.0, -0.5)}
UP_TYPE = (2, 4)
DOWN_TYPE = (1, 3, 5)


def chiral(kind, sw2):
    """(Q, g_L, g_R) of a fermion kind 'u', 'd' or 'l'."""
    q, t3 = CHARGES[kind]
    return q, t3 - q * sw2, -q * sw2


def chi(shat, mz, gz, sw2):
    """Z propagator relative to the photon's, with the coupling factor."""
    cw2 = 1.0 - sw2
    return shat / (sw2 * cw2 * (shat - mz * mz + 1j * mz * gz))


def m2bar(cos, shat, kind, alpha, mz, gz, sw2):
    """Spin- and colour-averaged |M|^2 of q qbar -> l- l+ (kind 'u' or 'd'),
    cos = cos(angle between the quark and the l-)."""
    qq, gq = chiral(kind, sw2)[0], chiral(kind, sw2)[1:]
    ql, gl = chiral("l", sw2)[0], chiral("l", sw2)[1:]
    x = chi(np.asarray(shat, dtype=np.float64), mz, gz, sw2)
    e4 = (4.0 * math.pi * alpha) ** 2
    cos = np.asarray(cos, dtype=np.float64)
    tot = 0.0
    for i in range(2):
        for j in range(2):
            f = qq * ql + gq[i] * gl[j] * x
            ang = (1.0 + cos) ** 2 if i == j else (1.0 - cos) ** 2
            tot = tot + ang * np.abs(f) ** 2
    return e4 / 12.0 * tot


def dsigma_dcos(cos, shat, kind, alpha, mz, gz, sw2):
    return m2bar(cos, shat, kind, alpha, mz, gz, sw2) / (32.0 * math.pi * shat)


def phase_space(u, sqrt_s, m_lo, m_hi):
    """(tau, y, cos) map of u (n, 3) over the mass window."""
    u = np.asarray(u, dtype=np.float64)
    s = sqrt_s * sqrt_s
    tlo, thi = m_lo * m_lo / s, m_hi * m_hi / s
    lr = math.log(thi / tlo)
    tau = tlo * np.exp(u[:, 0] * lr)
    ltau = np.log(1.0 / tau)
    y = (u[:, 1] - 0.5) * ltau
    cos = 2.0 * u[:, 2] - 1.0
    jac = (tau * lr) * ltau * 2.0
    sq = np.sqrt(tau)
    return dict(tau=tau, y=y, cos=cos, jac=jac, x1=sq * np.exp(y), x2=sq * np.exp(-y), shat=tau * s)


def integrand(u, grid, sqrt_s, m_lo, m_hi, alpha, mz, gz, sw2, gev2_to_pb):
    """F(u) in pb for u (n, 3)."""
    k = phase_space(u, sqrt_s, m_lo, m_hi)
    q2 = np.full(k["x1"].shape, mz * mz)
    f1 = pdf_oracle.interp(grid, k["x1"], q2)
    f2 = pdf_oracle.interp(grid, k["x2"], q2)
    tot = np.zeros_like(k["tau"])
    for q in (1, 2, 3, 4, 5):
        kind = "u" if q in UP_TYPE else "d"
        fwd = dsigma_dcos(k["cos"], k["shat"], kind, alpha, mz, gz, sw2)
        bwd = dsigma_dcos(-k["cos"], k["shat"], kind, alpha, mz, gz, sw2)
        tot = tot + f1[IDX[q]] * f2[IDX[-q]] * fwd + f1[IDX[-q]] * f2[IDX[q]] * bwd
    return k["jac"] / k["tau"] * tot * gev2_to_pb


def integrand_from_config(u, grid, c):
    return integrand(u, grid, c["sqrt_s"], c["m_lo"], c["m_hi"], c["alpha_em"], c["m_z"], c["gamma_z"], c["sw2"],
                     c["gev2_to_pb"])

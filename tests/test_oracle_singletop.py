"""Pins of the oracle's LO s-channel single-top integrand (u dbar -> t bbar)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import singletop as st, vegas
from oracle.pdf import interp
from oracle.ttbar import IDX
from synth import C6, synthetic_pdf_grid
from tests import dirac

MT, MW, GW, SW2, AL = C6["m_top"], C6["m_w"], C6["gamma_w"], C6["sw2"], C6["alpha_em"]

# W+ -> t bbar is fed by an up-type quark and a down-type antiquark of total
# charge +1; with a diagonal CKM matrix only same-generation pairs couple
CHARGE = {1: -1 / 3, 2: 2 / 3, 3: -1 / 3, 4: 2 / 3, 5: -1 / 3}
GENERATION = {1: 1, 2: 1, 3: 2, 4: 2, 5: 3}
W_PLUS_PAIRS = [(q, -qb) for q in (2, 4) for qb in (1, 3, 5)
                if abs(CHARGE[q] - CHARGE[qb] - 1) < 1e-12 and GENERATION[q] == GENERATION[qb]]


def m2_trace(p1, p2, p3, p4):
    """Spin- and colour-averaged |M|^2 of q(p1) qbar'(p2) -> t(p3) bbar(p4)
    from Dirac traces: spin average 1/4, colour sum N_c^2 over the average
    N_c^2 (two colour-singlet currents)."""
    s = (p1[0] + p2[0]) ** 2 - sum((p1[k] + p2[k]) ** 2 for k in (1, 2, 3))
    g = math.sqrt(4 * math.pi * AL / SW2)
    v = [dirac.vector_vertex(g / math.sqrt(2), dirac.PL)]
    return dirac.spin_sum(v, v, [1.0 / (s - MW * MW + 1j * MW * GW)], p1, p2, p3, p4, m3=MT) / 4.0


def test_pairs():
    assert W_PLUS_PAIRS == [(2, -1), (4, -3)]
    assert sorted(st.PAIRS) == sorted(W_PLUS_PAIRS)


def test_matrix_element_matches_dirac_traces():
    rng = np.random.default_rng(7)
    for rs in (175.0, 200.0, 350.0, 1000.0, 4000.0):
        for cos, phi in zip(rng.uniform(-1, 1, 3), rng.uniform(0, 2 * math.pi, 3)):
            ref = m2_trace(*dirac.cm_momenta(rs, cos, phi, MT))
            got = st.m2bar(cos, rs * rs, MT, MW, GW, SW2, AL)
            assert got == pytest.approx(ref, rel=1e-12)


def test_partonic_cross_section_textbook_form():
    for rs in (180.0, 250.0, 600.0, 3000.0):
        s = rs * rs
        num, _ = quad(lambda c: st.dsigma_dcos(c, s, MT, MW, GW, SW2, AL), -1, 1, epsabs=0, epsrel=1e-13)
        ref = math.pi * AL**2 / (24 * SW2**2) * (s - MT * MT) ** 2 * (2 * s + MT * MT) / (
            s * s * ((s - MW * MW) ** 2 + (MW * GW) ** 2))
        assert num == pytest.approx(ref, rel=1e-12)


def test_integrand_per_event_against_trace_assembly():
    grid = synthetic_pdf_grid()
    u = np.random.default_rng(3).uniform(0.02, 0.98, (6, 3))
    F = st.integrand_from_config(u, grid, C6)
    s = C6["sqrt_s"] ** 2
    tau0 = MT * MT / s
    for k in range(len(u)):
        tau = tau0 ** (1 - u[k, 0])
        y = (u[k, 1] - 0.5) * math.log(1 / tau)
        cos = 2 * u[k, 2] - 1
        x1, x2 = math.sqrt(tau) * math.exp(y), math.sqrt(tau) * math.exp(-y)
        f = interp(grid, np.array([x1, x2]), np.full(2, MT * MT))
        rs = math.sqrt(tau * s)
        fw = m2_trace(*dirac.cm_momenta(rs, cos, 0.7, MT, True))
        bw = m2_trace(*dirac.cm_momenta(rs, cos, 0.7, MT, False))
        tot = sum(f[IDX[q], 0] * f[IDX[qb], 1] * fw + f[IDX[qb], 0] * f[IDX[q], 1] * bw for q, qb in W_PLUS_PAIRS)
        beta = 1 - MT * MT / (tau * s)
        jac = tau * math.log(1 / tau0) * math.log(1 / tau) * 2
        ref = jac / tau * tot * beta / (32 * math.pi * tau * s) * C6["gev2_to_pb"]
        assert F[k] == pytest.approx(ref, rel=1e-11)


def test_hadronic_cross_section_vegas_vs_quadrature():
    """VEGAS on the oracle integrand against quadrature in (s_hat, y) of the
    luminosity times the textbook partonic cross section."""
    grid = synthetic_pdf_grid()
    s = C6["sqrt_s"] ** 2
    xg, wg = np.polynomial.legendre.leggauss(48)

    def sig(sh):
        return math.pi * AL**2 / (24 * SW2**2) * (sh - MT * MT) ** 2 * (2 * sh + MT * MT) / (
            sh * sh * ((sh - MW * MW) ** 2 + (MW * GW) ** 2))

    def dsig_dlntau(lt):
        tau = math.exp(lt)
        ly = math.log(1 / tau)
        ys = 0.5 * ly * xg
        x1, x2 = math.sqrt(tau) * np.exp(ys), math.sqrt(tau) * np.exp(-ys)
        f1 = interp(grid, x1, np.full(x1.shape, MT * MT))
        f2 = interp(grid, x2, np.full(x2.shape, MT * MT))
        lum = sum(0.5 * ly * np.sum(wg * (f1[IDX[q]] * f2[IDX[qb]] + f1[IDX[qb]] * f2[IDX[q]])) for q, qb in W_PLUS_PAIRS)
        # dtau = tau dln tau, and the 1/tau of f = xf/x
        return lum * sig(tau * s) * C6["gev2_to_pb"]

    ref, _ = quad(dsig_dlntau, math.log(MT * MT / s), 0.0, epsabs=0, epsrel=1e-9, limit=200)
    f = lambda u: st.integrand_from_config(u, grid, C6)
    res = vegas.run(f, 3, 50, 1.5, 5, 40000, seed=C6["seed"])
    assert abs(res["mean"] - ref) < 4 * res["sigma"]
    assert res["sigma"] / res["mean"] < 5e-3
    # LO s-channel single top at 8 TeV is a few pb; the synthetic PDFs land in the same range
    assert 0.5 < ref < 50.0

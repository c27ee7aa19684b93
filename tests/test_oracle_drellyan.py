"""Pins of the oracle's LO Drell-Yan integrand (q qbar -> gamma*/Z -> l+ l-)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import drellyan as dy, vegas
from oracle.pdf import interp
from oracle.ttbar import IDX
from synth import C5, synthetic_pdf_grid
from tests import dirac

AL, MZ, GZ, SW2 = C5["alpha_em"], C5["m_z"], C5["gamma_z"], C5["sw2"]

def _vertices(kind):
    """[photon, Z] vertex matrices for a fermion kind."""
    q, t3 = dy.CHARGES[kind]
    e = math.sqrt(4 * math.pi * AL)
    sw, cw = math.sqrt(SW2), math.sqrt(1 - SW2)
    gl, gr = t3 - q * SW2, -q * SW2
    return [dirac.vector_vertex(e * q), dirac.vector_vertex(e / (sw * cw), gl * dirac.PL + gr * dirac.PR)]


def m2_trace(p1, p2, p3, p4, kind):
    """Spin- and colour-averaged |M|^2 of q(p1) qbar(p2) -> l-(p3) l+(p4)
    from Dirac traces: spin average 1/4, colour N_c / N_c^2."""
    s = (p1[0] + p2[0]) ** 2 - sum((p1[k] + p2[k]) ** 2 for k in (1, 2, 3))
    props = [1.0 / s, 1.0 / (s - MZ * MZ + 1j * MZ * GZ)]
    return dirac.spin_sum(_vertices(kind), _vertices("l"), props, p1, p2, p3, p4) / 4.0 / 3.0


def _momenta(rs, cos, phi, quark_along_plus_z=True):
    return dirac.cm_momenta(rs, cos, phi, 0.0, quark_along_plus_z)


@pytest.mark.parametrize("kind", ["u", "d"])
def test_matrix_element_matches_dirac_traces(kind):
    rng = np.random.default_rng(11)
    for rs in (62.0, 85.0, MZ, 97.3, 119.0, 600.0):
        for cos, phi in zip(rng.uniform(-1, 1, 3), rng.uniform(0, 2 * math.pi, 3)):
            ref = m2_trace(*_momenta(rs, cos, phi), kind)
            got = dy.m2bar(cos, rs * rs, kind, AL, MZ, GZ, SW2)
            assert got == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("kind", ["u", "d"])
def test_photon_only_limit_is_qed(kind):
    q = dy.CHARGES[kind][0]
    for rs in (10.0, 70.0, 300.0):
        shat = rs * rs
        num, _ = quad(lambda c: dy.dsigma_dcos(c, shat, kind, AL, 1e9, GZ, SW2), -1, 1, epsabs=0, epsrel=1e-13)
        assert num == pytest.approx(4 * math.pi * AL**2 * q * q / (9 * shat), rel=1e-9)


def _width(kind, nc):
    q, gl, gr = dy.chiral(kind, SW2)
    return nc * AL * MZ * (gl * gl + gr * gr) / (6 * SW2 * (1 - SW2))


@pytest.mark.parametrize("kind", ["u", "d"])
def test_z_pole_is_photon_plus_breit_wigner_peak(kind):
    q = dy.CHARGES[kind][0]
    shat = MZ * MZ
    num, _ = quad(lambda c: dy.dsigma_dcos(c, shat, kind, AL, MZ, GZ, SW2), -1, 1, epsabs=0, epsrel=1e-13)
    ref = 4 * math.pi * AL**2 * q * q / (9 * shat) + 12 * math.pi * _width(kind, 3) * _width("l", 1) / (
        9 * MZ * MZ * GZ * GZ)
    assert num == pytest.approx(ref, rel=1e-12)
    # sanity of the width reading: Z -> nu nubar (T3 = 1/2, Q = 0) is about 166 MeV
    assert 0.160 < AL * MZ * 0.25 / (6 * SW2 * (1 - SW2)) < 0.172


def test_integrand_per_event_against_trace_assembly():
    """F(u) against a sum assembled from Dirac-trace |M|^2 with the quark
    from either beam, at the map's (x1, x2, cos)."""
    grid = synthetic_pdf_grid()
    u = np.random.default_rng(5).uniform(0.02, 0.98, (6, 3))
    F = dy.integrand_from_config(u, grid, C5)
    s = C5["sqrt_s"] ** 2
    tlo, thi = (C5["m_lo"] ** 2 / s), (C5["m_hi"] ** 2 / s)
    for k in range(len(u)):
        tau = tlo * (thi / tlo) ** u[k, 0]
        y = (u[k, 1] - 0.5) * math.log(1 / tau)
        cos = 2 * u[k, 2] - 1
        x1, x2 = math.sqrt(tau) * math.exp(y), math.sqrt(tau) * math.exp(-y)
        f = interp(grid, np.array([x1, x2]), np.full(2, MZ * MZ))
        rs = math.sqrt(tau * s)
        tot = 0.0
        for q in (1, 2, 3, 4, 5):
            kind = "u" if q in (2, 4) else "d"
            tot += f[IDX[q], 0] * f[IDX[-q], 1] * m2_trace(*_momenta(rs, cos, 0.3, True), kind)
            tot += f[IDX[-q], 0] * f[IDX[q], 1] * m2_trace(*_momenta(rs, cos, 0.3, False), kind)
        # dx1 dx2 = dtau dy, f = xf / x, d sigma / dcos = |M|^2 / (32 pi s_hat)
        jac = tau * math.log(thi / tlo) * math.log(1 / tau) * 2
        ref = jac / tau * tot / (32 * math.pi * tau * s) * C5["gev2_to_pb"]
        assert F[k] == pytest.approx(ref, rel=1e-11)


def test_hadronic_cross_section_vegas_vs_quadrature():
    """VEGAS on the oracle integrand against quadrature in (m_ll, y) of the
    luminosity times the angle-integrated partonic cross section."""
    grid = synthetic_pdf_grid()
    s = C5["sqrt_s"] ** 2
    xg, wg = np.polynomial.legendre.leggauss(48)
    sig_cache = {}

    def sigma_hat(shat, kind):
        key = (shat, kind)
        if key not in sig_cache:
            sig_cache[key] = float(np.sum(wg * dy.dsigma_dcos(xg, shat, kind, AL, MZ, GZ, SW2)))
        return sig_cache[key]

    def dsig_dm(m):
        tau = m * m / s
        ly = math.log(1 / tau)
        ys = 0.5 * ly * xg
        x1, x2 = math.sqrt(tau) * np.exp(ys), math.sqrt(tau) * np.exp(-ys)
        f1 = interp(grid, x1, np.full(x1.shape, MZ * MZ))
        f2 = interp(grid, x2, np.full(x2.shape, MZ * MZ))
        tot = 0.0
        for q in (1, 2, 3, 4, 5):
            kind = "u" if q in (2, 4) else "d"
            lum = 0.5 * ly * np.sum(wg * (f1[IDX[q]] * f2[IDX[-q]] + f1[IDX[-q]] * f2[IDX[q]]))
            tot += lum * sigma_hat(m * m, kind)
        # dtau = 2 m dm / s and the 1/tau of f = xf/x
        return tot / tau * 2 * m / s * C5["gev2_to_pb"]

    ref, _ = quad(dsig_dm, C5["m_lo"], C5["m_hi"], points=[MZ], epsabs=0, epsrel=1e-8, limit=200)
    f = lambda u: dy.integrand_from_config(u, grid, C5)
    res = vegas.run(f, 3, 50, 1.5, 5, 40000, seed=C5["seed"])
    assert abs(res["mean"] - ref) < 4 * res["sigma"]
    assert res["sigma"] / res["mean"] < 5e-3
    # LO Z/gamma* -> l l at 13 TeV in 60-120 GeV is O(2 nb); the synthetic PDFs land in the same range
    assert 200.0 < ref < 20000.0

"""Brute-force Dirac algebra for the matrix-element pins (test helper).

Explicit 4x4 gamma matrices (Dirac representation) and spin sums written as
traces: for a 2 -> 2 process a(p1) b(p2) -> c(p3) d(p4) with s-channel
currents vbar(p2) G_a u(p1) and ubar(p3) G'_a v(p4) summed over the exchanged
bosons a with propagator factors P_a,
  sum_spins |M|^2 = sum_{a,b} P_a P_b^* Tr[G_a^mu p1/ Gbar_b^rho p2/]
                                     Tr[G'_a,mu p4/ G'bar_b,rho (p3/ + m3)],
with Gbar = gamma^0 G^dagger gamma^0 and the metric lowering the indices.
"""
import numpy as np

_I2, _Z2 = np.eye(2), np.zeros((2, 2))
_SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
GAM = [np.block([[_I2, _Z2], [_Z2, -_I2]]).astype(complex)] + [np.block([[_Z2, s], [-s, _Z2]]) for s in _SIG]
G5 = 1j * GAM[0] @ GAM[1] @ GAM[2] @ GAM[3]
PL, PR = (np.eye(4) - G5) / 2, (np.eye(4) + G5) / 2
METRIC = np.array([1.0, -1.0, -1.0, -1.0])


def slash(p):
    return p[0] * GAM[0] - p[1] * GAM[1] - p[2] * GAM[2] - p[3] * GAM[3]


def bar(m):
    return GAM[0] @ m.conj().T @ GAM[0]


def vector_vertex(coupling, chiral=None):
    """[coupling gamma^mu chiral for mu = 0..3]; chiral defaults to 1."""
    c = np.eye(4) if chiral is None else chiral
    return [coupling * GAM[m] @ c for m in range(4)]


def spin_sum(vq, vf, props, p1, p2, p3, p4, m3=0.0):
    """sum over all spins of |M|^2 (real part; the imaginary part vanishes)."""
    s1, s2, s3, s4 = slash(p1), slash(p2), slash(p3) + m3 * np.eye(4), slash(p4)
    tot = 0.0 + 0.0j
    for a in range(len(props)):
        for b in range(len(props)):
            for mu in range(4):
                for rho in range(4):
                    hq = np.trace(vq[a][mu] @ s1 @ bar(vq[b][rho]) @ s2)
                    hf = np.trace(vf[a][mu] @ s4 @ bar(vf[b][rho]) @ s3)
                    tot += props[a] * np.conj(props[b]) * METRIC[mu] * METRIC[rho] * hq * hf
    assert abs(tot.imag) <= 1e-9 * abs(tot.real)
    return tot.real


def cm_momenta(rs, cos, phi, m3=0.0, incoming_along_plus_z=True):
    """Massless p1, p2 along -/+ z (p1 along +z unless flipped), p3 of mass m3
    at angle (theta, phi) with cos theta = cos, p4 massless, in the
    partonic rest frame of energy rs."""
    e = rs / 2.0
    sin = np.sqrt(1.0 - cos * cos)
    pa, pb = np.array([e, 0.0, 0.0, e]), np.array([e, 0.0, 0.0, -e])
    s = rs * rs
    pm = (s - m3 * m3) / (2.0 * rs)
    e3 = (s + m3 * m3) / (2.0 * rs)
    p3 = np.array([e3, pm * sin * np.cos(phi), pm * sin * np.sin(phi), pm * cos])
    p4 = np.array([pm, -p3[1], -p3[2], -p3[3]])
    return (pa, pb, p3, p4) if incoming_along_plus_z else (pb, pa, p3, p4)

"""RAMBO phase-space points and acceptance-rejection unweighting (oracle) —
test infrastructure.

Thesis: MC chapter (the RAMBO subsection: massless momenta from an isotropic,
q e^-q energy spectrum boosted and scaled to the total momentum, flat weight
w0; massive momenta by a common rescaling xi of the 3-momenta with weight
w0 w_m; the acceptance-rejection paragraph) and the MadFlow chapter (phase
space generation, unweighted event exporter: accept an event when its weight
exceeds a uniform number times the sample's largest weight).

Definitions implemented (P = (sqrt_s, 0, 0, 0), s = sqrt_s^2):
  per particle i, uniforms (u1, u2, u3, u4):
    c = 2 u1 - 1, phi = 2 pi u2, q0 = -ln(u3 u4),
    q = q0 (sqrt(1-c^2) cos phi, sqrt(1-c^2) sin phi, c);
  Q = sum q_i, M = sqrt(Q^2), b = -Q_vec/M, x = sqrt_s/M, gamma = Q0/M,
  a = 1/(1+gamma);
  p_i^0 = x (gamma q_i^0 + b.q_i),  p_i = x (q_i + b q_i^0 + a (b.q_i) b);
  w0 = (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / (Gamma(n) Gamma(n-1)).
  Massive: xi in (0, 1] with sum_i sqrt(m_i^2 + xi^2 (p_i^0)^2) = sqrt_s;
  k_i = (sqrt(m_i^2 + xi^2 (p_i^0)^2), xi p_i);
  w_m = s^(2-n) (sum |k_i|)^(2n-3) (prod |k_i|/k_i^0) / (sum |k_i|^2/k_i^0);
  the weight is w0 w_m (w0 alone when every mass is zero).
Readings: the printed massive energy sqrt(m^2 + (p^0)^2) omits xi, which
the constraint on xi that follows it requires; the sum over i = 1..k in w_m
runs over the n particles.  Random numbers: the uniforms of event e are
those of sample e of the VEGAS convention (philox.sample_uniforms with 4n
dimensions; particle i takes dimensions 4i..4i+3).  xi is found here by
bisection to the last bit (the kernel uses Newton's method).

Unweighting: with w_max the largest weight (or a given bound), event e is
kept when w_e > r_e w_max, r_e the first uniform of Philox block 0xFF of
sample e for the given (seed, stream, iteration) -- a block no sampler uses,
so the accept number is independent of the numbers that made the event;
kept indices in ascending order.

Pins: tests/test_oracle_rambo.py -- momentum conservation and mass shells;
the two- and three-body massless volumes 1/(8 pi) and s/(256 pi^3); the
massive two-body weight beta/(8 pi) event by event; the massive three-body
volume against a Dalitz-plot quadrature; the flat (Dirichlet) Dalitz
distribution of massless three-body points; isotropy; unweighting
acceptance rates and the unweighted distribution.
"""
import math

import numpy as np

from .philox import philox4x32, sample_uniforms, to_unit

UNWEIGHT_BLOCK = 0xFF  # Philox block field of the accept numbers (no sampler uses it)

UNWEIGHT_BLOCK = 0xFF  # Philox block field of the accept numbers (no sampler uses it)


def massless_weight(n, sqrt_s):
    """w0, the flat weight of n massless momenta (the phase-space volume)."""
    s = sqrt_s * sqrt_s
    return ((2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2)
            / (math.gamma(n) * math.gamma(n - 1)))


def massless_momenta(u, sqrt_s):
    """u (N, 4n) uniforms -> p (N, n, 4) massless momenta summing to P."""
    N = u.shape[0]
    n = u.shape[1] // 4
    uu = u.reshape(N, n, 4)
    c = 2.0 * uu[:, :, 0] - 1.0
    phi = 2.0 * math.pi * uu[:, :, 1]
    q0 = -np.log(uu[:, :, 2] * uu[:, :, 3])
    st = np.sqrt(1.0 - c * c)
    q = np.stack([q0, q0 * st * np.cos(phi), q0 * st * np.sin(phi), q0 * c], axis=2)
    Q = q[:, 0, :].copy()
    for i in range(1, n):
        Q = Q + q[:, i, :]
    M = np.sqrt(Q[:, 0] * Q[:, 0] - Q[:, 1] * Q[:, 1] - Q[:, 2] * Q[:, 2] - Q[:, 3] * Q[:, 3])
    b = -Q[:, 1:] / M[:, None]
    x = sqrt_s / M
    gam = Q[:, 0] / M
    a = 1.0 / (1.0 + gam)
    p = np.empty_like(q)
    for i in range(n):
        qi = q[:, i, :]
        bq = b[:, 0] * qi[:, 1] + b[:, 1] * qi[:, 2] + b[:, 2] * qi[:, 3]
        p[:, i, 0] = x * (gam * qi[:, 0] + bq)
        for j in range(3):
            p[:, i, j + 1] = x * (qi[:, j + 1] + b[:, j] * qi[:, 0] + a * bq * b[:, j])
    return p


def solve_xi(E, masses, sqrt_s):
    """xi per event (E: (N, n) massless energies) by bisection on (0, 1]."""
    m2 = np.asarray(masses, dtype=np.float64)[None, :] ** 2
    lo = np.zeros(E.shape[0])
    hi = np.ones(E.shape[0])
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = np.sqrt(m2 + (mid[:, None] * E) ** 2).sum(axis=1) - sqrt_s
        lo = np.where(f < 0.0, mid, lo)
        hi = np.where(f < 0.0, hi, mid)
        if np.all(hi - lo <= np.spacing(hi)):
            break
    return hi


def generate(seed, stream, iteration, first, n_events, masses, sqrt_s):
    """Momenta k (N, n, 4) and weights w (N,) of events first..first+N-1."""
    masses = np.asarray(masses, dtype=np.float64)
    n = masses.size
    u = sample_uniforms(seed, stream, iteration, np.arange(first, first + n_events, dtype=np.uint64), 4 * n)
    p = massless_momenta(u, sqrt_s)
    w0 = massless_weight(n, sqrt_s)
    if not np.any(masses > 0.0):
        return p, np.full(n_events, w0)
    xi = solve_xi(p[:, :, 0], masses, sqrt_s)
    k = np.empty_like(p)
    k[:, :, 0] = np.sqrt(masses[None, :] ** 2 + (xi[:, None] * p[:, :, 0]) ** 2)
    k[:, :, 1:] = xi[:, None, None] * p[:, :, 1:]
    kabs = xi[:, None] * p[:, :, 0]  # |k_i| = xi |p_i| = xi p_i^0 (massless p)
    s = sqrt_s * sqrt_s
    wm = (s ** (2 - n) * kabs.sum(axis=1) ** (2 * n - 3) * np.prod(kabs / k[:, :, 0], axis=1)
          / (kabs ** 2 / k[:, :, 0]).sum(axis=1))
    return k, w0 * wm


def unweight(w, seed, stream, iteration, w_max=None):
    """Ascending indices of the kept events and the w_max used."""
    w = np.asarray(w, dtype=np.float64)
    if w_max is None or w_max <= 0.0:
        w_max = float(np.max(np.where(w > 0.0, w, 0.0))) if w.size else 0.0
    # r_e: first word of Philox block 0xFF of sample e.  Sampling uses blocks
    # 0..(number of 4-word blocks it needs) - 1, so the accept number of an
    # event is never one of the numbers that made the event, whatever stream
    # and iteration the caller passes.
    idx = np.arange(w.size, dtype=np.uint64)
    lo = (idx & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    hi = (idx >> np.uint64(32)).astype(np.uint32)
    c3 = np.uint32(((stream << 8) | UNWEIGHT_BLOCK) & 0xFFFFFFFF)
    r = to_unit(philox4x32(lo, hi, np.uint32(iteration), c3, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)[0])
    return np.nonzero(w > r * w_max)[0], w_max

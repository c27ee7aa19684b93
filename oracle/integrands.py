"""Test integrands and their closed-form integrals (oracle) — test infrastructure.

  gauss      prod_j N(x_j; c_j, s_j), each factor normalised on the real line;
             over [0,1]^d its integral is
             prod_j (erf((1-c_j)/(s_j sqrt2)) + erf(c_j/(s_j sqrt2)))/2.
  genz_osc   cos(2 pi w_1 + sum_i c_i x_i), integral
             Re[ e^{i 2 pi w_1} prod_j (e^{i c_j} - 1)/(i c_j) ]   (Genz 1984).
  genz_peak  prod_i (c_i^-2 + (x_i - w_i)^2)^-1, integral
             prod_i c_i [atan(c_i (1 - w_i)) + atan(c_i w_i)]      (Genz 1984).

The closed forms are exact integrals; they are the pins of the Monte Carlo
estimators (tests compare sampled means with them within a few sigma, and
low-dimensional product quadrature with them to rounding).
"""
import math

import numpy as np

GAUSS, GENZ_OSC, GENZ_PEAK = 0, 1, 2


def gauss(x, centre, sigma):
    x = np.asarray(x, dtype=np.float64)
    c = np.broadcast_to(np.asarray(centre, dtype=np.float64), (x.shape[1],))
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (x.shape[1],))
    z = (x - c) / s
    norm = np.prod(1.0 / (s * math.sqrt(2.0 * math.pi)))
    return norm * np.exp(-0.5 * np.sum(z * z, axis=1))


def gauss_integral(dim, centre, sigma):
    c = np.broadcast_to(np.asarray(centre, dtype=np.float64), (dim,))
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (dim,))
    val = 1.0
    for cj, sj in zip(c, s):
        val *= 0.5 * (math.erf((1.0 - cj) / (sj * math.sqrt(2.0))) + math.erf(cj / (sj * math.sqrt(2.0))))
    return val


def genz_osc(x, w1, c):
    x = np.asarray(x, dtype=np.float64)
    return np.cos(2.0 * math.pi * w1 + x @ np.asarray(c, dtype=np.float64))


def genz_osc_integral(w1, c):
    z = complex(math.cos(2.0 * math.pi * w1), math.sin(2.0 * math.pi * w1))
    for cj in c:
        z *= (complex(math.cos(cj), math.sin(cj)) - 1.0) / complex(0.0, cj)
    return z.real


def genz_peak(x, w, c):
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    return np.prod(1.0 / (c ** -2 + (x - w) ** 2), axis=1)


def genz_peak_integral(w, c):
    val = 1.0
    for wj, cj in zip(w, c):
        val *= cj * (math.atan(cj * (1.0 - wj)) + math.atan(cj * wj))
    return val


def from_params(kind, dim, params):
    """Return (f, exact integral) for a batched-workload parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    if kind == GAUSS:
        c, s = p[:dim], p[dim:2 * dim]
        return (lambda x: gauss(x, c, s)), gauss_integral(dim, c, s)
    if kind == GENZ_OSC:
        w1, c = p[0], p[1:1 + dim]
        return (lambda x: genz_osc(x, w1, c)), genz_osc_integral(w1, c)
    if kind == GENZ_PEAK:
        w, c = p[:dim], p[dim:2 * dim]
        return (lambda x: genz_peak(x, w, c)), genz_peak_integral(w, c)
    raise ValueError(kind)

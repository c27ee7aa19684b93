"""Pins of the Genz closed forms (oscillatory, product peak) in the oracle.

The batched workload's integrals of these families are compared with
genz_osc_integral and genz_peak_integral.  Here those closed forms are checked
against product Gauss-Legendre quadrature of the integrands themselves over the
full d-dimensional tensor grid (d = 1, 2, 3), not against a second copy of the
formula: a wrong sign, a dropped factor or a swapped parameter in either the
integrand or its closed form shows up as a difference far above 1e-12.

Genz (1984), "Testing multidimensional integration routines": oscillatory
f = cos(2 pi w_1 + sum c_i x_i), product peak f = prod (c_i^-2 + (x_i - w_i)^2)^-1.
The quadrature is composite (P panels of n nodes per axis), so the nearest
complex singularity of the product peak (x = w_i +- i/c_i) lies many panel
widths' worth of Bernstein ellipse away and the rule is exact to rounding.
"""
import itertools

import numpy as np
import pytest

from oracle.integrands import genz_osc, genz_osc_integral, genz_peak, genz_peak_integral
from synth.batch import GENZ_OSC, GENZ_PEAK, batch_specs


def composite_gauss_legendre(panels, n):
    """Nodes and weights of a composite Gauss-Legendre rule on [0, 1]."""
    t, w = np.polynomial.legendre.leggauss(n)
    h = 1.0 / panels
    xs = np.concatenate([(k + 0.5 * (t + 1.0)) * h for k in range(panels)])
    ws = np.concatenate([0.5 * h * w for _ in range(panels)])
    return xs, ws


def tensor_quadrature(f, dim, panels, n):
    """sum over the full tensor grid of prod_j w_j f(x), in slabs."""
    x1, w1 = composite_gauss_legendre(panels, n)
    m = x1.size
    total = 0.0
    # the first axis is looped over so that a slab holds m^(dim-1) points
    rest = [np.array(p) for p in zip(*itertools.product(range(m), repeat=dim - 1))] if dim > 1 else []
    for i0 in range(m):
        if dim == 1:
            pts = np.array([[x1[i0]]])
            wts = np.array([w1[i0]])
        else:
            cols = [np.full(rest[0].size, x1[i0])] + [x1[r] for r in rest]
            pts = np.stack(cols, axis=1)
            wts = w1[i0] * np.prod(np.stack([w1[r] for r in rest], axis=1), axis=1)
        total += float(np.dot(wts, f(pts)))
    return total


def _rule_is_converged(f, dim):
    """The tensor rule at two resolutions agrees to rounding (so its value is
    the integral, not a resolution artefact)."""
    a = tensor_quadrature(f, dim, 4, 24)
    b = tensor_quadrature(f, dim, 6, 24)
    return a, b


OSC_CASES = [
    (0.0, [1.0]),
    (0.37, [4.5]),
    (0.81, [0.3, 2.2]),
    (0.12, [2.5, 2.0]),
    (0.55, [1.0, 2.0, 1.5]),
    (0.9, [0.2, 0.3, 4.0]),
]
PEAK_CASES = [
    ([0.5], [7.25]),
    ([0.1], [3.0]),
    ([0.3, 0.8], [5.0, 2.25]),
    ([0.95, 0.02], [1.0, 6.25]),
    ([0.2, 0.5, 0.7], [2.0, 3.0, 2.25]),
    ([0.9, 0.4, 0.05], [0.5, 4.5, 2.25]),
]


@pytest.mark.parametrize("w1,c", OSC_CASES)
def test_genz_oscillatory_closed_form_against_quadrature(w1, c):
    dim = len(c)
    f = lambda x: genz_osc(x, w1, c)
    a, b = _rule_is_converged(f, dim)
    assert abs(a - b) <= 1e-13
    # integrand bounded by 1 on the unit cube: an absolute bar
    assert abs(genz_osc_integral(w1, c) - b) <= 1e-12


@pytest.mark.parametrize("w,c", PEAK_CASES)
def test_genz_product_peak_closed_form_against_quadrature(w, c):
    dim = len(c)
    f = lambda x: genz_peak(x, w, c)
    a, b = _rule_is_converged(f, dim)
    assert abs(a - b) <= 1e-13 * abs(b)
    assert genz_peak_integral(w, c) == pytest.approx(b, rel=1e-12, abs=0)


def test_batched_workload_genz_members_against_quadrature():
    """The low-dimensional Genz members of the seeded batched workload (the
    parameters the GPU batch is actually checked with) against quadrature."""
    checked = 0
    for spec in batch_specs(n_integrals=400):
        if spec.dim > 3 or spec.kind not in (GENZ_OSC, GENZ_PEAK):
            continue
        d, p = spec.dim, spec.params
        if spec.kind == GENZ_OSC:
            w1, c = p[0], p[1:1 + d]
            q = tensor_quadrature(lambda x: genz_osc(x, w1, c), d, 6, 24)
            assert abs(genz_osc_integral(w1, c) - q) <= 1e-12
        else:
            w, c = p[:d], p[d:2 * d]
            q = tensor_quadrature(lambda x: genz_peak(x, w, c), d, 6, 24)
            assert genz_peak_integral(w, c) == pytest.approx(q, rel=1e-12, abs=0)
        checked += 1
    assert checked >= 4


def test_planted_mistakes_are_caught():
    """A sign slip in the oscillatory phase or a missing factor c in the
    peak's closed form (plausible mistakes) moves the value far beyond the
    bar, so the quadrature comparison above would catch them."""
    w1, c = 0.37, [1.3, 2.1]
    q = tensor_quadrature(lambda x: genz_osc(x, w1, c), 2, 6, 24)
    z = complex(np.cos(2 * np.pi * w1), -np.sin(2 * np.pi * w1))  # conjugated phase
    for cj in c:
        z *= (complex(np.cos(cj), np.sin(cj)) - 1.0) / complex(0.0, cj)
    assert abs(z.real - q) > 1e-3
    w, cc = [0.3, 0.8], [5.0, 2.25]
    q = tensor_quadrature(lambda x: genz_peak(x, w, cc), 2, 6, 24)
    wrong = np.prod([np.arctan(ci * (1 - wi)) + np.arctan(ci * wi) for wi, ci in zip(w, cc)])
    assert abs(wrong - q) > 1e-3 * abs(q)

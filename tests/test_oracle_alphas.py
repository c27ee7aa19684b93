"""Pins of the oracle's alpha_s(Q) interpolation."""
import numpy as np
import pytest

from oracle import alphas as oa
from synth import synthetic_pdf_grid, synthetic_alphas
from synth.alphas import AlphasTable, alphas_exact


@pytest.fixture(scope="module")
def table():
    return synthetic_alphas(synthetic_pdf_grid())


def test_node_values_exact(table):
    for s, (q, v) in enumerate(zip(table.q2_knots, table.values)):
        got = oa.interp(table, q)
        if s < len(table.q2_knots) - 1:
            # the top knot of a lower subgrid belongs to the next subgrid; the
            # table is continuous there
            assert np.allclose(got, v, rtol=1e-15, atol=0)
        else:
            assert np.array_equal(got, v)


def test_quadratics_reproduced_on_uniform_subgrids(table):
    rng = np.random.default_rng(0)
    for s, q in enumerate(table.q2_knots):
        b = np.log(q)
        assert np.allclose(np.diff(b), np.diff(b)[0], rtol=1e-12)  # uniform in ln Q^2
    coef = (0.3, -0.02, 0.004)
    quad = lambda b: coef[0] + coef[1] * b + coef[2] * b * b
    t = AlphasTable(table.q2_knots, [quad(np.log(q)) for q in table.q2_knots])
    for s, q in enumerate(table.q2_knots):
        if len(q) < 4:
            continue
        lo, hi = np.log(q[1]), np.log(q[-2])  # interior cells: full stencil
        bb = rng.uniform(lo, hi, 200)
        assert np.allclose(oa.interp(t, np.exp(bb)), quad(bb), rtol=1e-13, atol=1e-15)


def test_linear_functions_everywhere(table):
    lin = lambda b: 0.2 - 0.01 * b
    t = AlphasTable(table.q2_knots, [lin(np.log(q)) for q in table.q2_knots])
    q2 = np.exp(np.random.default_rng(1).uniform(np.log(table.q2_knots[0][0]), np.log(table.q2_knots[-1][-1]), 500))
    assert np.allclose(oa.interp(t, q2), lin(np.log(q2)), rtol=1e-13, atol=1e-15)


def test_outside_the_table(table):
    top, bottom = table.q2_knots[-1][-1], table.q2_knots[0][0]
    assert np.all(oa.interp(table, [top * 1.5, top * 100]) == table.values[-1][-1])
    assert np.all(np.isnan(oa.interp(table, [bottom * 0.9, 0.0])))


def test_one_loop_function_within_interpolation_error(table):
    """Error against the sampled function: O(h^3) in the cubic cells, O(h^2)
    (about h^2 |f''|/8 with h = 0.6 in ln Q^2) in the linear edge cells."""
    q2 = np.exp(np.random.default_rng(2).uniform(np.log(table.q2_knots[0][0]), np.log(1e10), 4000))
    rel = np.abs(oa.interp(table, q2) / alphas_exact(q2) - 1)
    edge = np.zeros(q2.shape, dtype=bool)
    for q in table.q2_knots:
        edge |= ((q2 >= q[0]) & (q2 < q[1])) | ((q2 >= q[-2]) & (q2 <= q[-1]))
    assert rel[~edge].max() < 2e-4
    assert rel[edge].max() < 3e-3
    # alpha_s(M_Z) = 0.118 is the anchor of the table
    assert oa.interp(table, [91.1876**2])[0] == pytest.approx(0.118, rel=1e-5)

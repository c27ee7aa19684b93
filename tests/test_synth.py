"""Sanity of the seeded synthetic inputs (no GPU)."""
import numpy as np

from synth import C1, C3, FLAVOURS, batch_specs, pdf_queries, synthetic_pdf_grid, he_init_segments
from synth.pdfgrid import momentum_sum_at_q0


def test_grid_shape_and_thresholds():
    g = synthetic_pdf_grid()
    assert len(g.x_knots) == 196 and g.x_knots[0] == 1e-9 and g.x_knots[-1] == 1.0
    assert np.all(np.diff(np.log(g.x_knots)) > 0)
    assert [len(q) for q in g.q2_knots] == [4, 12, 34]
    assert sum(len(q) for q in g.q2_knots) == 50
    assert g.q2_knots[0][-1] == g.q2_knots[1][0] == 1.3 ** 2
    assert g.q2_knots[1][-1] == g.q2_knots[2][0] == 4.75 ** 2
    assert g.q2_knots[2][-1] == 1e10
    for s, vals in enumerate(g.xf):
        assert vals.shape == (11, len(g.q2_knots[s]), 196)
        for fi, pid in enumerate(FLAVOURS):
            zero = (abs(pid) == 4 and s < 1) or (abs(pid) == 5 and s < 2)
            assert np.all(vals[fi] == 0.0) == zero
    assert momentum_sum_at_q0(g) == np.float64(momentum_sum_at_q0(g))
    assert abs(momentum_sum_at_q0(g) - 1.0) < 1e-14


def test_grid_is_deterministic():
    a, b = synthetic_pdf_grid(), synthetic_pdf_grid()
    for va, vb in zip(a.xf, b.xf):
        assert np.array_equal(va, vb)


def test_queries_in_range():
    x, q2 = pdf_queries(100_000)
    assert x.min() >= C1["x_min"] and x.max() <= C1["x_max"]
    assert q2.min() >= C1["query_q_min"] ** 2 and q2.max() <= C1["query_q_max"] ** 2


def test_batch_specs_ranges():
    specs = batch_specs()
    assert len(specs) == C3["n_integrals"]
    for s in specs:
        assert C3["dim_min"] <= s.dim <= C3["dim_max"]
        assert C3["n_min"] * 0.99 <= s.n <= C3["n_max"] * 1.01
    assert {s.kind for s in specs} == {0, 1, 2}
    assert [s.stream for s in specs] == list(range(len(specs)))


def test_he_init_segments():
    p = he_init_segments([("w", 4, 256), ("b", 4, 64), ("z", 64, 128)], seed=3)
    assert p.dtype == np.float32 and p.size == 448
    assert np.all(p[256:] == 0.0)
    assert abs(np.std(p[:256]) - np.sqrt(2 / 4)) < 0.15


def test_pdf_replicas():
    from synth import C7, synthetic_pdf_replicas, fk_points
    g = synthetic_pdf_grid()
    a = synthetic_pdf_replicas(g, 4, C7["eps"], C7["seed"])
    b = synthetic_pdf_replicas(g, 4, C7["eps"], C7["seed"])
    assert len(a) == 4 and all(len(m) == len(g.xf) for m in a)
    for ma, mb in zip(a, b):
        for va, vb, v0 in zip(ma, mb, g.xf):
            assert np.array_equal(va, vb) and va.shape == v0.shape
            assert np.array_equal(va == 0.0, v0 == 0.0)  # zeros stay zeros
            nz = v0 != 0.0
            assert np.all(np.abs(va[nz] / v0[nz] - 1.0) < 0.5)
    assert not np.array_equal(a[0][2], a[1][2])
    x, q2 = fk_points(C7)
    assert x.size == 2415 and np.all(np.diff(x) > 0) and np.all(q2 == 1.65 ** 2)
    assert g.q2_knots[1][0] < q2[0] < g.q2_knots[1][-1]

"""Batched persistent VEGAS (one graph per iteration) vs the single-integral
path, the oracle and the closed forms."""
import math

import numpy as np
import pytest

from oracle import vegas as ov
from oracle.integrands import from_params
from oracle.philox import sample_uniforms
from synth import batch_specs, C3

pytestmark = pytest.mark.gpu


def ctx_for(vgx, spec, seed, prec=None):
    prec = vgx.F32 if prec is None else prec
    return vgx.vegas_create(spec.kind, spec.dim, C3["n_bins"], C3["alpha"], seed, spec.stream, prec, spec.params)


@pytest.mark.parametrize("tile,block", [(0, 0), (256, 64), (3000, 128)])
def test_batch_equals_single_integral_path(vgx, tile, block):
    print(f"batch vs single tile={tile} block={block}", flush=True)
    specs = batch_specs(n_integrals=10, n_scale=0.01, seed=7)
    seed = 99
    A = [ctx_for(vgx, s, seed) for s in specs]
    B = [ctx_for(vgx, s, seed) for s in specs]
    try:
        b = vgx.batch_create(A, [s.n for s in specs], tile, block)
        try:
            t, bl = vgx.batch_config(b)
            if tile:
                assert (t, bl) == (tile, block)
            for it in range(3):
                rb = vgx.batch_iterate(b, it, len(specs))
                for k, s in enumerate(specs):
                    rs = vgx.vegas_iterate(B[k], s.n, it)
                    vgx.vegas_refine(B[k])
                    scale = math.sqrt(s.n * rs["s2"]) + abs(rs["s1"])
                    assert abs(rb[k]["s1"] - rs["s1"]) <= 1e-12 * scale
                    assert rb[k]["s2"] == pytest.approx(rs["s2"], rel=1e-12)
                    assert rb[k]["n"] == s.n
            for k, s in enumerate(specs):
                ea = vgx.vegas_get_grid(A[k], s.dim, C3["n_bins"])
                eb = vgx.vegas_get_grid(B[k], s.dim, C3["n_bins"])
                assert np.max(np.abs(ea - eb)) < 1e-12
                ra, rb2 = vgx.vegas_result(A[k]), vgx.vegas_result(B[k])
                assert ra["n_used"] == 3 and ra["mean"] == pytest.approx(rb2["mean"], rel=1e-10, abs=1e-12)
        finally:
            vgx.batch_destroy(b)
    finally:
        for c in A + B:
            vgx.vegas_destroy(c)


def test_batch_first_iteration_matches_oracle(vgx):
    specs = batch_specs(n_integrals=6, n_scale=0.005, seed=11)
    ctxs = [ctx_for(vgx, s, 5) for s in specs]
    try:
        b = vgx.batch_create(ctxs, [s.n for s in specs], 0, 0)
        try:
            res = vgx.batch_iterate(b, 0, len(specs))
        finally:
            vgx.batch_destroy(b)
        for k, s in enumerate(specs):
            f, _ = from_params(s.kind, s.dim, s.params)
            ref = ov.iteration(f, ov.uniform_grid(s.dim, C3["n_bins"]), 5, s.stream, 0, s.n)
            w = ref["w"]
            # FP32 integrand: per-sample relative error <~ 1e-6, absolute for
            # the oscillatory family
            tol = 1e-5 * math.fsum(np.abs(w))
            assert abs(res[k]["s1"] - ref["s1"]) <= tol
            h = vgx.vegas_get_hist(ctxs[k], s.dim, C3["n_bins"])
            assert np.allclose(h, ref["hist"], rtol=3e-5, atol=1e-6 * ref["s2"])
    finally:
        for c in ctxs:
            vgx.vegas_destroy(c)


def test_full_batched_workload_against_closed_forms(vgx):
    """The batched workload (64 integrals, d 2..12, 1e4..1e7 samples,
    10 iterations in one graph replay each): every integral agrees with
    its closed form, and the pulls are standard-normal-like."""
    print("batched workload 64 integrals x 10 iterations", flush=True)
    specs = batch_specs()
    ctxs = [ctx_for(vgx, s, C3["seed"]) for s in specs]
    try:
        b = vgx.batch_create(ctxs, [s.n for s in specs], 0, 0)
        try:
            for it in range(C3["iterations"]):
                vgx.batch_iterate(b, it, len(specs))
        finally:
            vgx.batch_destroy(b)
        pulls = []
        for k, s in enumerate(specs):
            _, I = from_params(s.kind, s.dim, s.params)
            r = vgx.vegas_result(ctxs[k])
            assert r["n_used"] == C3["iterations"]
            # FP32 integrand bias bound ~1e-6 relative
            pulls.append((r["mean"] - I) / math.hypot(r["sigma"], 1e-6 * abs(I)))
        pulls = np.array(pulls)
        print(f"  pulls mean {pulls.mean():.2f} std {pulls.std():.2f} max {np.abs(pulls).max():.2f}")
        assert np.all(np.abs(pulls) < 5.0)
        assert abs(pulls.mean()) < 0.6
        assert 0.5 < pulls.std() < 1.6
    finally:
        for c in ctxs:
            vgx.vegas_destroy(c)


def test_batch_rejects_bad_input(vgx, pdf_ctx):
    s = batch_specs(n_integrals=1, n_scale=0.001)[0]
    c = ctx_for(vgx, s, 1)
    try:
        with pytest.raises(vgx.VgxError):
            vgx.batch_create([c, c], [s.n, s.n])
        with pytest.raises(vgx.VgxError):
            vgx.batch_create([c], [1])
        t = vgx.vegas_create(vgx.TTBAR, 3, 50, 1.5, 0, 0, vgx.F32, np.array([13000.0, 173.0, 0.118, 3.893793721e8]),
                             pdf=pdf_ctx)
        try:
            with pytest.raises(vgx.VgxError):
                vgx.batch_create([c, t], [s.n, 100])
        finally:
            vgx.vegas_destroy(t)
    finally:
        vgx.vegas_destroy(c)


@pytest.mark.parametrize("big_bins", [110, 256])
def test_batch_with_large_histograms(vgx, big_bins):
    """Histograms too large for four LDS copies per workgroup: 12 x 110 bins
    takes two copies, 12 x 256 one; sums, histograms and refined grids still
    equal those of the single-integral path."""
    print(f"batch with a 12 x {big_bins} histogram", flush=True)
    shapes = [(12, big_bins, 40_000), (2, 50, 30_000), (5, 77, 25_001)]

    def make_ctx(k, d, nb):
        params = np.concatenate([np.full(d, 0.45), np.full(d, 0.25)])
        return vgx.vegas_create(vgx.GAUSS, d, nb, 1.5, 31, 40 + k, vgx.F32, params)

    A = [make_ctx(k, d, nb) for k, (d, nb, _) in enumerate(shapes)]
    B = [make_ctx(k, d, nb) for k, (d, nb, _) in enumerate(shapes)]
    try:
        b = vgx.batch_create(A, [n for _, _, n in shapes], 0, 0)
        try:
            for it in range(3):
                rb = vgx.batch_iterate(b, it, len(shapes))
                for k, (d, nb, n) in enumerate(shapes):
                    rs = vgx.vegas_iterate(B[k], n, it)
                    hb, hs = vgx.vegas_get_hist(A[k], d, nb), vgx.vegas_get_hist(B[k], d, nb)
                    assert np.allclose(hb, hs, rtol=1e-12, atol=0.0)
                    vgx.vegas_refine(B[k])
                    assert rb[k]["s1"] == pytest.approx(rs["s1"], rel=1e-12)
                    assert rb[k]["s2"] == pytest.approx(rs["s2"], rel=1e-12)
            for k, (d, nb, _) in enumerate(shapes):
                ea, eb = vgx.vegas_get_grid(A[k], d, nb), vgx.vegas_get_grid(B[k], d, nb)
                assert np.max(np.abs(ea - eb)) < 1e-12
        finally:
            vgx.batch_destroy(b)
    finally:
        for c in A + B:
            vgx.vegas_destroy(c)

"""Checkpoint/resume, per-estimate tracing and allocation-failure paths.

Resume: the iteration's random numbers are counter-based (sample index,
iteration index, stream, key), so an iteration depends only on its grid and
its counters.  A run stopped after k iterations, its grid saved with
vegas_get_grid and loaded into a fresh context with vegas_set_grid, then
continued with the same iteration indices, must give bit-identical records
and grids to the uninterrupted run.

Tracing: VGX_TRACE names a file that every estimate read back is appended
to as one JSON line; the lines must carry exactly the records vegas_results
returns, and the grid hash must change exactly when the grid does.

Allocation failures: VGX_FAIL_ALLOC=k makes the k-th allocation (counted
from the variable's last change) fail; every create must then return
VGX_ENOMEM with its message set, leave nothing behind (the device's free
memory is unchanged after many such failures), and work again once the
variable is cleared.
"""
import json
import os

import numpy as np
import pytest

from synth import C2, he_init_segments

pytestmark = pytest.mark.gpu


def _gauss_ctx(vgx, seed=7):
    prm = np.concatenate([np.full(4, 0.5), np.full(4, 0.1)])
    return vgx.vegas_create(vgx.GAUSS, 4, 50, 1.5, seed, 2, vgx.F64, prm)


def _run(vgx, v, its, n):
    recs = []
    for it in its:
        recs.append(vgx.vegas_iterate(v, n, it))
        vgx.vegas_refine(v)
    return recs


def test_resume_from_saved_grid_is_bit_identical(vgx):
    print("resume: 10 iterations against 5 + save/load + 5", flush=True)
    n = 200_003
    a = _gauss_ctx(vgx)
    b = _gauss_ctx(vgx)
    c = _gauss_ctx(vgx)
    try:
        ra = _run(vgx, a, range(10), n)
        _run(vgx, b, range(5), n)
        grid = vgx.vegas_get_grid(b, 4, 50)
        vgx.vegas_set_grid(c, grid)
        rc = _run(vgx, c, range(5, 10), n)
        for x, y in zip(ra[5:], rc):
            for k in ("mean", "var", "s1", "s2", "n"):
                assert x[k] == y[k], (k, x[k], y[k])
        assert np.array_equal(vgx.vegas_get_grid(a, 4, 50), vgx.vegas_get_grid(c, 4, 50))
    finally:
        for v in (a, b, c):
            vgx.vegas_destroy(v)


def test_trace_lines_match_the_records(vgx, tmp_path, monkeypatch):
    path = tmp_path / "trace.jsonl"
    monkeypatch.setenv("VGX_TRACE", str(path))
    v = _gauss_ctx(vgx, seed=11)
    try:
        recs = []
        for it in range(4):
            recs.append(vgx.vegas_iterate(v, 100_000, it))
            if it != 1:  # no refinement after iteration 1: iteration 2 samples the same grid
                vgx.vegas_refine(v)
        monkeypatch.delenv("VGX_TRACE")
        vgx.vegas_iterate(v, 100_000, 9)  # not traced
        lines = [json.loads(x) for x in path.read_text().splitlines()]
        assert len(lines) == 4
        for k, (line, r) in enumerate(zip(lines, recs)):
            assert line["record"] == k and line["kind"] == "plain" and line["finite"] == 1
            assert line["n"] == r["n"] and line["mean"] == r["mean"] and line["var"] == r["var"]
        hashes = [line["grid_fnv1a"] for line in lines]
        assert hashes[1] == hashes[2] and len({hashes[0], hashes[1], hashes[3]}) == 3
        res = vgx.vegas_result(v)
        assert lines[-1]["records_used"] == 4 and np.isfinite(lines[-1]["combined_sigma"])
        assert res["mean"] != 0.0
    finally:
        vgx.vegas_destroy(v)


def _free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_injected_allocation_failures_return_enomem_and_leak_nothing(vgx, c1_grid, monkeypatch):
    prm = np.concatenate([np.full(4, 0.5), np.full(4, 0.1)])
    params = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])
    pdf = vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf)
    init = he_init_segments(vgx.flow_param_layout(3), 1)
    makers = {
        "vegas": (lambda: vgx.vegas_create(vgx.GAUSS, 4, 50, 1.5, 1, 0, vgx.F64, prm), vgx.vegas_destroy),
        "vegas_ttbar": (lambda: vgx.vegas_create(vgx.TTBAR, 3, 50, 1.5, 1, 0, vgx.F32, params, pdf=pdf),
                        vgx.vegas_destroy),
        "flow": (lambda: vgx.flow_create(3, init), vgx.flow_destroy),
        "pdf": (lambda: vgx.pdf_create(c1_grid.x_knots, c1_grid.q2_knots, c1_grid.xf), vgx.pdf_destroy),
    }
    try:
        for name, (make, destroy) in makers.items():
            # warm: the first create may set up runtime state of its own
            destroy(make())
            before = _free_bytes()
            failures = 0
            for rep in range(3):
                for k in range(1, 40):
                    monkeypatch.setenv("VGX_FAIL_ALLOC", str(k))
                    try:
                        obj = make()
                    except vgx.VgxError as e:
                        assert e.status == vgx.VGX_ENOMEM and "VGX_FAIL_ALLOC" in str(e), str(e)
                        failures += 1
                        continue
                    finally:
                        monkeypatch.setenv("VGX_FAIL_ALLOC", "")
                    destroy(obj)  # k beyond this create's allocations: it succeeded
            monkeypatch.delenv("VGX_FAIL_ALLOC")
            after = _free_bytes()
            print(f"  {name}: {failures // 3} allocation points failed and recovered; free memory "
                  f"{before} -> {after}", flush=True)
            assert failures >= 3
            assert before - after < (8 << 20), (name, before, after)
            destroy(make())  # works again
    finally:
        vgx.pdf_destroy(pdf)


def test_kernel_timing_samples_one_launch_in_k(vgx):
    """vegas_set_timing(every=k) brackets launches 0, k, 2k, ... after the
    call; vegas_kernel_time returns their count and summed duration."""
    v = _gauss_ctx(vgx, seed=3)
    try:
        for every, n_launch, timed in ((1, 7, 7), (3, 10, 4), (4, 8, 2)):
            vgx.vegas_set_timing(v, True, every=every)
            for it in range(n_launch):
                vgx.vegas_iterate_async(v, 200_000, it)
            ms, launches = vgx.vegas_kernel_time(v)
            print(f"  every={every}: {launches} timed launches, {ms / max(launches, 1):.4f} ms each", flush=True)
            assert launches == timed and ms > 0.0
        vgx.vegas_set_timing(v, False)
        vgx.vegas_iterate_async(v, 1000, 99)
        assert vgx.vegas_kernel_time(v)[1] == 0
        with pytest.raises(vgx.VgxError):
            vgx._check(vgx._c["vegas_set_timing"](v, -1), "vegas_set_timing")
    finally:
        vgx.vegas_destroy(v)


def test_deferred_records_match_synchronous_iterations(vgx):
    """vegas_iterate_async leaves its record holding S1 and S2 only; the next
    refinement completes it in a workgroup of its own, and every other call
    that reads or adds records completes it first.  A context driven through
    each of those routes must hold, bit for bit, the records, combination
    and grid of one driven by vegas_iterate."""
    import torch
    print("deferred records: async routes against synchronous iterations", flush=True)
    n = 150_001
    a, b = _gauss_ctx(vgx, seed=21), _gauss_ctx(vgx, seed=21)
    ba = bb = None

    def same(where, grids=True):
        ra, rb = vgx.vegas_results(a), vgx.vegas_results(b)
        assert len(ra) == len(rb), where
        for k, (x, y) in enumerate(zip(ra, rb)):
            for key in ("mean", "var", "s1", "s2", "n"):
                assert x[key] == y[key], (where, k, key, x[key], y[key])
        ca, cb = vgx.vegas_result(a), vgx.vegas_result(b)
        assert ca == cb, (where, ca, cb)
        if grids:
            assert np.array_equal(vgx.vegas_get_grid(a, 4, 50), vgx.vegas_get_grid(b, 4, 50)), where

    try:
        # completed by the refinement's extra workgroup
        vgx.vegas_iterate(a, n, 0); vgx.vegas_refine(a)
        vgx.vegas_iterate_async(b, n, 0); vgx.vegas_refine(b)
        same("refine")
        # completed by the next iteration (no refinement in between)
        vgx.vegas_iterate(a, n, 1)
        vgx.vegas_iterate_async(b, n, 1)
        vgx.vegas_iterate(a, n, 2); vgx.vegas_refine(a)
        vgx.vegas_iterate_async(b, n, 2); vgx.vegas_refine(b)
        same("next iteration")
        # completed by the readbacks
        vgx.vegas_iterate(a, n, 3)
        vgx.vegas_iterate_async(b, n, 3)
        assert vgx.vegas_result(a) == vgx.vegas_result(b)
        vgx.vegas_iterate(a, n, 4)
        vgx.vegas_iterate_async(b, n, 4)
        same("results")
        # completed before caller points are estimated
        y = torch.rand((4, 100_003), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
        vgx.vegas_iterate(a, n, 5)
        vgx.vegas_iterate_async(b, n, 5)
        pa = vgx.vegas_iterate_points(a, y)
        pb = vgx.vegas_iterate_points(b, y)
        assert pa["mean"] == pb["mean"] and pa["var"] == pb["var"]
        same("points")
        # completed before a batched iteration of the context
        vgx.vegas_iterate(a, n, 6)
        vgx.vegas_iterate_async(b, n, 6)
        ba = vgx.batch_create([a], [n])
        bb = vgx.batch_create([b], [n])
        assert vgx.batch_iterate(ba, 7, 1) == vgx.batch_iterate(bb, 7, 1)
        # the batch refines too, from histograms summed by LDS atomics in an
        # order that varies from run to run: its grids agree only to rounding
        same("batch", grids=False)
        ga, gb = vgx.vegas_get_grid(a, 4, 50), vgx.vegas_get_grid(b, 4, 50)
        assert np.allclose(ga, gb, rtol=0, atol=1e-12)
        vgx.vegas_set_grid(b, ga)
        # a pending record is discarded with the others
        vgx.vegas_iterate(a, n, 8)
        vgx.vegas_iterate_async(b, n, 8)
        vgx.vegas_reset_results(a)
        vgx.vegas_reset_results(b)
        assert len(vgx.vegas_results(b)) == 0 and vgx.vegas_result(b)["n_used"] == 0
        vgx.vegas_iterate(a, n, 9); vgx.vegas_refine(a)
        vgx.vegas_iterate_async(b, n, 9); vgx.vegas_refine(b)
        same("reset")
        assert len(vgx.vegas_results(b)) == 1
    finally:
        for bt in (ba, bb):
            if bt is not None:
                vgx.batch_destroy(bt)
        vgx.vegas_destroy(a)
        vgx.vegas_destroy(b)

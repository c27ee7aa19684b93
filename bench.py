"""Benchmark of the VEGAS hot path on one MI355X.

Workload (the headline): LO pp -> t tbar at sqrt(s) = 13 TeV, 3-d
(tau, y, cos theta*) integrand with log-bicubic PDF interpolation on the
synthetic 11-flavour grid and closed-form LO |M|^2; VEGAS with 50 bins per
dimension, 1e7 events per iteration, FP32 integrand with FP64 map and
compensated FP64 sums.

One step = one pass of the hot path over one batch: Philox uniforms, grid
map with Jacobians, fused integrand (PDF interpolation x |M|^2), per-bin
histograms and compensated sums, fixed-order reduction, estimate and
inverse-variance combination, grid refinement.  Inputs (PDF grid, VEGAS
grid) are resident in HBM before the timed region.

Also reported: the fused kernel's roofline (FP32 VALU; kernel time from HIP
events on the stream it runs on), the FP64 oracle timed on a bounded
sample on the host cores, and the time to 1e-4 relative error of plain
VEGAS and of the flow-proposal pipeline when available.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s + time to 1e-4 rel. error: plain VEGAS vs flow sampler, 1 MI355X"

# Algorithmic FP32 flops per t tbar event of the fused kernel: per x value
# the 4x4 Hermite stencil for 11 flavours (16 weights + 176 FMA = 368 flops)
# plus ~32 flops of cell/basis setup, twice (x1, x2), plus ~60 flops of
# kinematics, matrix elements and luminosities.
FLOPS_PER_EVENT_F32 = 2 * (368 + 32) + 60
PEAK_FP32 = 157.3e12     # MI355X FP32 vector (packed) peak
PEAK_FP32_UNPACKED = 78.6e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=None, help="events per iteration (default 1e7)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-flow", action="store_true", help="skip the flow comparison")
    return ap.parse_args()


def cpu_baseline(grid, n_sample):
    """The FP64 oracle on the first n_sample events of iteration 0 (uniform
    grid), timed on the host.  Returns events/s."""
    import numpy as np
    from oracle import ttbar as ot, vegas as ov
    from oracle.philox import sample_uniforms
    from synth import C2
    e = ov.uniform_grid(3, C2["n_bins"])
    t0 = time.perf_counter()
    u = sample_uniforms(C2["seed"], 0, 0, np.arange(n_sample, dtype=np.uint64), 3)
    x, jac, idx = ov.vegas_map(u, e)
    w = ot.integrand(x, grid, C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]) * jac
    ov.estimate_from_weights(w, idx, 3, C2["n_bins"])
    dt = time.perf_counter() - t0
    return n_sample / dt, dt


def time_to_precision_vegas(vgx, pdf, params, n_iter_events, target=1e-4, max_iter=30):
    """Plain VEGAS from a uniform grid until sigma/mean <= target."""
    import torch
    from synth import C2
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], 1000 + C2["seed"], 0, vgx.F32, params, pdf=pdf)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = 0
        res = None
        while it < max_iter:
            vgx.vegas_iterate(v, n_iter_events, it)
            vgx.vegas_refine(v)
            res = vgx.vegas_result(v)
            it += 1
            if res["sigma"] <= target * abs(res["mean"]):
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dict(seconds=dt, iterations=it, events=it * n_iter_events, mean=res["mean"], sigma=res["sigma"],
                    reached=bool(res["sigma"] <= target * abs(res["mean"])))
    finally:
        vgx.vegas_destroy(v)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2302_03343_amd.vgx as vgx
    from synth import C2, synthetic_pdf_grid

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    grid = synthetic_pdf_grid()
    pdf = vgx.pdf_create(grid.x_knots, grid.q2_knots, grid.xf)
    params = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])
    n = args.events or C2["n_per_iter"]
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], C2["seed"], 0, vgx.F32, params, pdf=pdf)

    it = 0
    for _ in range(args.warmup):
        vgx.vegas_iterate(v, n, it)
        vgx.vegas_refine(v)
        it += 1
    torch.cuda.synchronize()
    vgx.vegas_set_timing(v, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        vgx.vegas_iterate(v, n, it)
        vgx.vegas_refine(v)
        it += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = vgx.vegas_kernel_time(v)
    vgx.vegas_set_timing(v, False)
    res = vgx.vegas_result(v)
    vgx.vegas_destroy(v)

    ms_per_step = dt / args.steps * 1e3
    value = n * args.steps / dt
    kern_avg_s = kern_ms / max(launches, 1) * 1e-3
    achieved = FLOPS_PER_EVENT_F32 * n / kern_avg_s
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "LO pp->ttbar 13 TeV, VEGAS 3-d, 50 bins/dim, 1e7 events/iteration, "
                        "log-bicubic PDF (synthetic 11-flavour grid, 196 x, 3 Q subgrids), "
                        "FP32 integrand, FP64 map and compensated sums",
            "events_per_iteration": n,
            "sigma_pb": res["sigma"], "mean_pb": res["mean"], "chi2_dof": res["chi2_dof"],
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "frac_of_unpacked_fp32": achieved / PEAK_FP32_UNPACKED,
            "traffic": None,
            "kernel": "k_vegas_iter<3,TTbar,PhiloxSrc<3>,true>",
            "kernel_avg_ms": kern_avg_s * 1e3,
            "flops_per_event": FLOPS_PER_EVENT_F32,
            "events_per_launch": n,
        },
    }
    if not args.no_flow:
        out["time_to_1e-4"] = {"vegas": time_to_precision_vegas(vgx, pdf, params, n)}
    if not args.no_cpu:
        n_cpu = 300_000
        eps, secs = cpu_baseline(grid, n_cpu)
        out["cpu_baseline"] = {"value": eps, "unit": "events/s", "cores": 1, "kind": "oracle",
                               "sample": f"first {n_cpu} events of iteration 0 (uniform grid), FP64 numpy, "
                                         f"{secs:.1f} s"}
    vgx.pdf_destroy(pdf)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

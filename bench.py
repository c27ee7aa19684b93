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

# Algorithmic FP32 flops per t tbar event of the fused kernel as built: per x
# value the tensor-product weights of the 4x4 Hermite stencil (16 products)
# shared by the 11 flavours, whose values are 11 x 16 FMA (352 flops), plus
# ~32 flops of cell and basis setup, twice (x1, x2), plus ~60 flops of
# kinematics, matrix elements and luminosities: 860.  Counting each
# flavour's 2-d stencil separately (four 1-d Hermites in x and one in Q^2,
# with slopes, ~50 flops a flavour) gives the ~1.3k of a per-flavour
# evaluation; the line reports both, the figure as built first.
FLOPS_PER_EVENT_F32 = 2 * (368 + 32) + 60
FLOPS_PER_EVENT_PER_FLAVOUR_COUNT = 1300
PEAK_FP32 = 157.3e12     # MI355X FP32 vector (packed) peak
PEAK_FP32_UNPACKED = 78.6e12

# HBM bytes per launch of the headline kernel, from the FETCH_SIZE/WRITE_SIZE
# passes summarised in this file; used only while the kernel's sources still
# hash to the digest recorded there (else the traffic is reported as null).
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ttbar_lo_1e7_counters.md")


def _profile_fields(path):
    fields = {}
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith("- ") and ": " in line:
                    k, v = line[2:].split(": ", 1)
                    fields[k.strip()] = v.strip()
    except OSError:
        pass
    return fields


def measured_traffic(events_per_launch):
    """Scaled HBM bytes per launch recorded for the current kernel sources,
    or None when the record is missing, stale or for another launch size."""
    import hashlib
    f = _profile_fields(TRAFFIC_PROFILE)
    try:
        srcs = f["sources"].split()
        h = hashlib.sha256()
        for s in srcs:
            with open(os.path.join(ROOT, s), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != f["source_sha256"] or int(f["events_per_launch"]) != events_per_launch:
            return None
        return float(f["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


EXTRA_NAMES = ("ttbar_fixed_scale_contraction", "ttbar_dynamic_scale", "drell_yan_1e7", "single_top_s_1e7",
               "pdf_interp_1e8", "vegas_gauss4_f64", "batched_64", "events", "pdf_members_fk_2415",
               "flow_train_ttbar", "flow_sample_ttbar")


def extras_table(vgx, pdf, grid, params, n):
    """The extra workloads by name, each a function of no arguments."""
    return {"ttbar_fixed_scale_contraction": lambda: extra_ttbar_contracted(vgx, pdf, params, n),
            "ttbar_dynamic_scale": lambda: extra_ttbar_dynamic(vgx, pdf, grid, params, n),
            "drell_yan_1e7": lambda: extra_drellyan(vgx, pdf, n),
            "single_top_s_1e7": lambda: extra_singletop(vgx, pdf, n),
            "pdf_interp_1e8": lambda: extra_pdf(vgx, pdf),
            "vegas_gauss4_f64": lambda: extra_gauss(vgx),
            "batched_64": lambda: extra_batch(vgx),
            "events": lambda: extra_events(vgx),
            "pdf_members_fk_2415": lambda: extra_members(vgx, grid),
            "flow_train_ttbar": lambda: extra_flow_train(vgx, pdf, params),
            "flow_sample_ttbar": lambda: extra_flow_sample(vgx, pdf, params, n)}


def _ttbar_flow_setup(vgx, pdf, params):
    """A t tbar context after one refinement and a coupling flow (d = 3) with
    He-normal hidden layers and a zero output layer."""
    from synth import C2, C4, he_init_segments
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], 1000 + C2["seed"], 0, vgx.F32, params, pdf=pdf)
    vgx.vegas_iterate(v, 1_000_000, 0)
    vgx.vegas_refine(v)
    f = vgx.flow_create(3, he_init_segments(vgx.flow_param_layout(3), C4["seed"]))
    return v, f


def extra_flow_train(vgx, pdf, params, steps=50):
    """Training steps of the d = 3 flow on t tbar samples of the refined grid
    (batch 1e5, lr 1e-3): milliseconds per step (training kernels alone, HIP
    events around the loop, data drawn beforehand)."""
    import torch
    from synth import C4
    v, f = _ttbar_flow_setup(vgx, pdf, params)
    try:
        n = C4["batch"]
        u = torch.empty((steps, 3, n), dtype=torch.float64, device="cuda")
        g = torch.empty((steps, n), dtype=torch.float64, device="cuda")
        for s in range(steps):
            vgx.vegas_sample(v, 0, n, 10_000 + s, u=u[s], g=g[s])
        vgx.flow_train_step(f, u[0], g[0], C4["lr"])  # first use allocates the training buffers
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for s in range(1, steps):
            vgx.flow_train_step(f, u[s], g[s], C4["lr"], sync=False)
        e1.record()
        e1.synchronize()
        loss = vgx.flow_train_step(f, u[0], g[0], 0.0)
        return {"ms_per_step": e0.elapsed_time(e1) / (steps - 1), "batch": n, "loss_after": loss}
    finally:
        vgx.flow_destroy(f)
        vgx.vegas_destroy(v)


def extra_flow_sample(vgx, pdf, params, n):
    """Flow points and their evaluation (weights f/q) for n t tbar events:
    milliseconds for the pair of calls (HIP events)."""
    import torch
    v, f = _ttbar_flow_setup(vgx, pdf, params)
    try:
        y = torch.empty((3, n), dtype=torch.float64, device="cuda")
        lq = torch.empty(n, dtype=torch.float64, device="cuda")
        vgx.flow_sample(f, n, 1, 5, 0, y, lq)
        vgx.vegas_iterate_points(v, y, lq)
        ms = cuda_timed(lambda: (vgx.flow_sample(f, n, 1, 5, 0, y, lq), vgx.vegas_iterate_points(v, y, lq)))
        return {"ms": ms, "ns_per_event": ms * 1e6 / n}
    finally:
        vgx.flow_destroy(f)
        vgx.vegas_destroy(v)


def one_extra(name, n_events):
    """One extra workload alone (for profiling its kernels)."""
    import numpy as np
    from paper_2302_03343_amd import vgx
    from synth import C2, synthetic_pdf_grid
    grid = synthetic_pdf_grid()
    pdf = vgx.pdf_create(grid.x_knots, grid.q2_knots, grid.xf)
    params = np.array([C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]])
    try:
        res = extras_table(vgx, pdf, grid, params, n_events or C2["n_per_iter"])[name]()
        print(json.dumps({"workload": name, name: res}), flush=True)
    finally:
        vgx.pdf_destroy(pdf)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    # the GPU's clocks take some 100 steps of sustained load (about 25 ms) to
    # settle; a short warm-up times the ramp instead of the kernel
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--events", type=int, default=None, help="events per iteration (default 1e7)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-flow", action="store_true", help="skip the flow comparison")
    ap.add_argument("--no-compact", action="store_true",
                    help="skip the compact figures of the other configurations (C0, C1, C3, C4 d = 8)")
    ap.add_argument("--extras", action="store_true",
                    help="also measure the other workloads (PDF interpolation alone, plain Gaussian VEGAS, "
                         "batched integrals) as extra fields")
    ap.add_argument("--pdf-only", action="store_true",
                    help="only the PDF interpolation workload (1e8 queries, FP64 and FP32 outputs); one JSON line")
    ap.add_argument("--extra", choices=EXTRA_NAMES, default=None,
                    help="only the named extra workload (for profiling its kernels); one JSON line")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only run a plain 2 GiB device copy (reference for scaling HBM counters) and exit")
    return ap.parse_args()


def _oracle_weights(grid, first, count, chunk):
    """FP64 oracle weights f J of events first .. first+count-1 of iteration
    0 on the uniform grid (the headline's counters), in chunks."""
    import numpy as np
    from oracle import ttbar as ot, vegas as ov
    from oracle.philox import sample_uniforms
    from synth import C2
    e = ov.uniform_grid(3, C2["n_bins"])
    out = []
    for s0 in range(first, first + count, chunk):
        idx_s = np.arange(s0, min(s0 + chunk, first + count), dtype=np.uint64)
        u = sample_uniforms(C2["seed"], 0, 0, idx_s, 3)
        x, jac, idx = ov.vegas_map(u, e)
        w = ot.integrand(x, grid, C2["sqrt_s"], C2["m_top"], C2["alpha_s"], C2["gev2_to_pb"]) * jac
        ov.estimate_from_weights(w, idx, 3, C2["n_bins"])   # sums and histograms, as an iteration does
        out.append(w)
    return np.concatenate(out)


def _oracle_range(args):
    """Worker of the P-core leg: one contiguous range of sample indices."""
    from threadpoolctl import threadpool_limits
    from synth import synthetic_pdf_grid
    first, count, chunk = args
    grid = synthetic_pdf_grid()
    with threadpool_limits(limits=1):
        _oracle_weights(grid, first, count, chunk)
    return count


def cpu_baseline(n_sample, chunk=250_000):
    """The FP64 oracle on the first n_sample events of iteration 0 (uniform
    grid): on one host core (library thread pools held to one thread), and
    over P worker processes splitting the sample-index range (P = the
    process's CPU affinity, at most 16, the host share of one GPU).  Runs
    before anything touches the GPU, so the workers are plain forks.
    Returns the figures and the oracle's S1, S2 (exact sums, math.fsum)."""
    import math
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from synth import synthetic_pdf_grid
    grid = synthetic_pdf_grid()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        w = _oracle_weights(grid, 0, n_sample, chunk)
        dt1 = time.perf_counter() - t0
    s1, s2 = math.fsum(w), math.fsum(w * w)
    P = max(1, min(16, len(os.sched_getaffinity(0))))
    share = (n_sample + P - 1) // P
    jobs = [(k * share, min(share, n_sample - k * share), min(chunk, share)) for k in range(P) if k * share < n_sample]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(len(jobs)) as pool:
        done = sum(pool.map(_oracle_range, jobs))
    dtp = time.perf_counter() - t0
    assert done == n_sample
    return dict(eps_1=n_sample / dt1, secs_1=dt1, eps_p=n_sample / dtp, secs_p=dtp, procs=len(jobs), s1=s1, s2=s2)


def next_batch(res, rel_var, target, n_max, n_min=100_000):
    """Samples for the next iteration or batch: the number that brings the
    inverse-variance combination to sigma/|mean| = target if the new batch
    has relative variance rel_var per sample (n var(E)/E^2 of the last
    batch), with 5 % margin, clamped to [n_min, n_max]."""
    mean, sigma = abs(res["mean"]), res["sigma"]
    if not (mean > 0 and sigma > 0 and rel_var > 0 and math.isfinite(rel_var)):
        return n_max
    need_inv_var = 1.0 / (target * mean) ** 2 - 1.0 / sigma ** 2
    if need_inv_var <= 0:
        return n_min
    n = int(math.ceil(1.05 * need_inv_var * rel_var * mean ** 2))
    return max(n_min, min(n_max, n))


def time_to_precision_vegas(vgx, pdf, params, n_iter_events, target=1e-4, max_iter=30, kind=None, dim=3,
                            seed=None):
    """Plain VEGAS from a uniform grid until sigma/mean <= target; the size
    of an iteration is the configured one, or less when fewer samples
    reach the target (the same rule as the flow pipeline's batches)."""
    import torch
    from synth import C2
    kind = vgx.TTBAR if kind is None else kind
    prec = vgx.F32 if kind == vgx.TTBAR else vgx.F64
    seed = 1000 + C2["seed"] if seed is None else seed
    v = vgx.vegas_create(kind, dim, C2["n_bins"], C2["alpha"], seed, 0, prec, params, pdf=pdf)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = 0
        res = None
        n_next, events = n_iter_events, 0
        while it < max_iter:
            r = vgx.vegas_iterate(v, n_next, it)
            vgx.vegas_refine(v)
            res = vgx.vegas_result(v)
            it += 1
            events += n_next
            if res["sigma"] <= target * abs(res["mean"]):
                break
            n_next = next_batch(res, r["var"] * r["n"] / r["mean"] ** 2, target, n_iter_events)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dict(seconds=dt, iterations=it, events=events, mean=res["mean"], sigma=res["sigma"],
                    reached=bool(res["sigma"] <= target * abs(res["mean"])))
    finally:
        vgx.vegas_destroy(v)


def flow_pipeline(vgx, kind, dim, params, pdf, n_iter, warm_iters, steps, batch, lr, n_flow, seed, target=1e-4,
                  max_batches=40):
    """Flow-proposal pipeline until sigma/mean <= target: VEGAS warm-up
    iterations (kept in the combination), training of the coupling flow on
    uniform points of the VEGAS cube with g = f(G(u)) J(u), then batches
    drawn from the flow (weights f/q) until the target is reached.  One
    warm-up iteration is used: measured on the t tbar integrand, the flow
    trained on the once-refined grid reaches a lower variance per sample
    (0.018) than on a twice-refined one (0.045).
    Wall time includes everything from the first launch."""
    import torch
    from synth import he_init_segments
    prec = vgx.F32 if kind == vgx.TTBAR else vgx.F64
    v = vgx.vegas_create(kind, dim, 50, 1.5, seed, 0, prec, params, pdf=pdf)
    init = he_init_segments(vgx.flow_param_layout(dim), seed)
    f = vgx.flow_create(dim, init)
    try:
        u = torch.empty((dim, batch), dtype=torch.float64, device="cuda")
        g = torch.empty(batch, dtype=torch.float64, device="cuda")
        ybuf = torch.empty(dim * n_flow, dtype=torch.float64, device="cuda")
        y = ybuf.view(dim, n_flow)
        lq = torch.empty(n_flow, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last_vegas = None
        for it in range(warm_iters):
            last_vegas = vgx.vegas_iterate(v, n_iter, it)
            vgx.vegas_refine(v)
        t_warm = time.perf_counter()
        losses = []
        for s in range(steps):
            vgx.vegas_sample(v, 0, batch, 10_000 + s, u=u, g=g)
            sync = (s == 0 or s == steps - 1)
            l = vgx.flow_train_step(f, u, g, lr, sync=sync)
            if sync:
                losses.append(l)
        torch.cuda.synchronize()
        t_train = time.perf_counter()
        k = 0
        res = vgx.vegas_result(v)
        last_flow = None
        # first flow batch: a pilot of n_flow/10 samples; then batches sized
        # from the flow's measured variance per sample
        n_next, flow_events = max(n_flow // 10, 1), 0
        while res["sigma"] > target * abs(res["mean"]) and k < max_batches:
            yk = ybuf[:dim * n_next].view(dim, n_next)
            vgx.flow_sample(f, n_next, seed, 5, k, yk, lq[:n_next])
            last_flow = vgx.vegas_iterate_points(v, yk, lq[:n_next])
            res = vgx.vegas_result(v)
            flow_events += n_next
            k += 1
            n_next = next_batch(res, last_flow["var"] * last_flow["n"] / last_flow["mean"] ** 2, target, n_flow)
        torch.cuda.synchronize()
        t_end = time.perf_counter()
        out = dict(seconds=t_end - t0, seconds_excluding_training=(t_end - t0) - (t_train - t_warm),
                   training_seconds=t_train - t_warm, warmup_iterations=warm_iters, train_steps=steps,
                   train_batch=batch, flow_batches=k, flow_events=flow_events, mean=res["mean"], sigma=res["sigma"],
                   reached=bool(res["sigma"] <= target * abs(res["mean"])), loss_first=losses[0],
                   loss_last=losses[-1])
        # --- after the timed pipeline: the samplers compared per sample and
        # per unit of time.  relvar = n var(E) / E^2 of the weights.
        rv = lambda r: r["var"] * r["n"] / r["mean"] ** 2
        out["rel_var_per_sample_vegas_uniform_grid"] = rv(last_vegas) if last_vegas else None
        if last_flow:
            out["rel_var_per_sample_flow"] = rv(last_flow)
        # cost per event of the flow: sampling and evaluating its points
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        vgx.flow_sample(f, n_flow, seed, 6, 0, y, lq)
        vgx.vegas_iterate_points(v, y, lq)
        e1.record()
        e1.synchronize()
        out["flow_ns_per_event"] = e0.elapsed_time(e1) * 1e6 / n_flow
        # the same in one pass (flow_vegas_iterate: no points in memory)
        e0.record()
        vgx.flow_vegas_iterate(f, v, n_flow, seed, 6, 1, allow_fallback=True)
        e1.record()
        e1.synchronize()
        out["flow_fused_ns_per_event"] = e0.elapsed_time(e1) * 1e6 / n_flow
        # the identity-initialised flow draws the VEGAS map's own points: one
        # fused iteration on the grid the flow was trained on measures it (a
        # fresh context, so the pipeline's combination is untouched)
        v2 = vgx.vegas_create(kind, dim, 50, 1.5, seed + 1, 0, prec, params, pdf=pdf)
        try:
            vgx.vegas_set_grid(v2, vgx.vegas_get_grid(v, dim, 50))
            vgx.vegas_set_timing(v2, True)
            vgx.vegas_iterate_async(v2, n_flow, 0)
            km, launches = vgx.vegas_kernel_time(v2)
            r2 = vgx.vegas_results(v2)[0]
        finally:
            vgx.vegas_destroy(v2)
        out["rel_var_per_sample_vegas_refined_grid"] = rv(r2)
        out["vegas_ns_per_event"] = km / launches * 1e6 / n_flow
        if last_flow:
            out["gain_trained_vs_identity_flow"] = rv(r2) / rv(last_flow)
            # sigma reached in equal wall time (training excluded), flow / VEGAS
            out["equal_wall_time_sigma_ratio_flow_over_vegas"] = math.sqrt(
                rv(last_flow) * out["flow_ns_per_event"] / (rv(r2) * out["vegas_ns_per_event"]))
        return out
    finally:
        vgx.flow_destroy(f)
        vgx.vegas_destroy(v)


def pdf_only():
    """The PDF interpolation workload alone (for profiling its kernel)."""
    from paper_2302_03343_amd import vgx
    from synth import synthetic_pdf_grid
    grid = synthetic_pdf_grid()
    pdf = vgx.pdf_create(grid.x_knots, grid.q2_knots, grid.xf)
    try:
        print(json.dumps({"workload": "pdf-logbicubic-11flav, 1e8 log-uniform queries",
                          "pdf_interp_1e8": extra_pdf(vgx, pdf)}), flush=True)
    finally:
        vgx.pdf_destroy(pdf)


def copy_reference():
    """A plain device-to-device copy of a known size; its FETCH_SIZE and
    WRITE_SIZE readings scale the counters of the measured kernels."""
    import torch
    n = 1 << 28  # 2 GiB of FP64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_reference_bytes": n * 8}), flush=True)


def cuda_timed(fn, reps=5):
    """Median milliseconds of fn() between HIP events on the current stream."""
    import torch
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def extra_pdf(vgx, pdf):
    """PDF interpolation alone: 1e8 log-uniform queries, FP64 and FP32 outputs."""
    import torch
    from synth import C1, pdf_queries
    n = C1["n_queries"]
    x, q2 = pdf_queries(n)
    xt, qt = torch.from_numpy(x).cuda(), torch.from_numpy(q2).cuda()
    del x, q2
    out = {}
    for name, dt, obytes in (("f64", torch.float64, 88), ("f32", torch.float32, 44)):
        res = torch.empty((11, n), dtype=dt, device="cuda")
        vgx.pdf_interp(pdf, xt, qt, res)
        ms = cuda_timed(lambda: vgx.pdf_interp(pdf, xt, qt, res))
        byt = n * (16 + obytes)
        out[name] = {"queries_per_s": n / (ms * 1e-3), "ms": ms, "algorithmic_GBps": byt / (ms * 1e-3) / 1e9,
                     "frac_of_8TBps": byt / (ms * 1e-3) / 8e12, "bytes_per_query": 16 + obytes}
        del res
    torch.cuda.empty_cache()
    return out


def extra_gauss(vgx):
    """Plain VEGAS on the d=4 Gaussian: the small configuration (10 x 1e5)
    and a chip-filling 1e9 samples per iteration."""
    import numpy as np
    from synth import C0
    prm = np.concatenate([np.full(4, C0["centre"]), np.full(4, C0["sigma"])])
    out = {}
    v = vgx.vegas_create(vgx.GAUSS, 4, C0["n_bins"], C0["alpha"], C0["seed"], 0, vgx.F64, prm)
    try:
        t0 = time.perf_counter()
        for it in range(C0["iterations"]):
            vgx.vegas_iterate(v, C0["n_per_iter"], it)
            vgx.vegas_refine(v)
        dt = time.perf_counter() - t0
        r = vgx.vegas_result(v)
        out["small"] = {"events_per_s": C0["iterations"] * C0["n_per_iter"] / dt, "ms_total": dt * 1e3,
                        "mean": r["mean"], "sigma": r["sigma"]}
        n = C0["n_per_iter_large"]
        vgx.vegas_set_timing(v, True)
        t0 = time.perf_counter()
        for it in range(3):
            vgx.vegas_iterate(v, n, 100 + it)
            vgx.vegas_refine(v)
        dt = time.perf_counter() - t0
        ms, k = vgx.vegas_kernel_time(v)
        kern = ms / k * 1e-3
        flops = 65.0 * n / kern
        out["large"] = {"events_per_s": 3 * n / dt, "kernel_ms": kern * 1e3, "fp64_flops_per_sample": 65,
                        "achieved_TFLOPs": flops / 1e12, "frac_of_fp64_peak": flops / 78.6e12}
    finally:
        vgx.vegas_destroy(v)
    return out


def extra_hadronic(vgx, pdf, kind, params, seed, n, k=10):
    """k GPU-resident iterations of n events of a fused hadronic integrand
    after 3 adaptation iterations: events/s and the fused kernel's time."""
    import torch
    from synth import C2
    v = vgx.vegas_create(kind, 3, C2["n_bins"], C2["alpha"], seed, 0, vgx.F32, params, pdf=pdf)
    try:
        for it in range(3):
            vgx.vegas_iterate(v, n, it)
            vgx.vegas_refine(v)
        torch.cuda.synchronize()
        vgx.vegas_set_timing(v, True)
        t0 = time.perf_counter()
        for it in range(k):
            vgx.vegas_iterate_async(v, n, 3 + it)
            vgx.vegas_refine(v)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, launches = vgx.vegas_kernel_time(v)
        r = vgx.vegas_result(v)
        return {"events_per_s": n * k / dt, "kernel_ms": ms / launches, "mean_pb": r["mean"], "sigma_pb": r["sigma"]}
    finally:
        vgx.vegas_destroy(v)


def extra_ttbar_contracted(vgx, pdf, params, n):
    """The same t tbar iteration with the Q^2 direction of the PDF stencil
    contracted once per workgroup at the fixed scale (mode 1)."""
    import numpy as np
    from synth import C2
    return extra_hadronic(vgx, pdf, vgx.TTBAR, np.concatenate([params, [1.0]]), C2["seed"], n)


def extra_ttbar_dynamic(vgx, pdf, grid, params, n):
    """The same t tbar workload with the scale set per event, mu^2 = s_hat/4,
    and running alpha_s(mu) (mode 2): the full per-event 2-d stencil."""
    import numpy as np
    from synth import C2, synthetic_alphas
    table = synthetic_alphas(grid)
    vgx.pdf_set_alphas(pdf, table.q2_knots, table.values)
    return extra_hadronic(vgx, pdf, vgx.TTBAR, np.concatenate([params, [2.0]]), C2["seed"], n)


def extra_singletop(vgx, pdf, n):
    """LO s-channel single top (u dbar, c sbar -> t bbar) at 8 TeV, the
    thesis's own LO example, on the same fused path (full stencil)."""
    import numpy as np
    from synth import C6
    p = np.array([C6["sqrt_s"], C6["m_top"], C6["m_w"], C6["gamma_w"], C6["sw2"], C6["alpha_em"], C6["gev2_to_pb"],
                  0.0])
    return extra_hadronic(vgx, pdf, vgx.SINGLETOP, p, C6["seed"], n)


def extra_drellyan(vgx, pdf, n):
    """LO Drell-Yan (photon/Z -> l+ l-, 60 < m_ll < 120 GeV) on the same fused
    path: full stencil (mode 0) and fixed-scale contraction (mode 1)."""
    import numpy as np
    from synth import C5
    p = np.array([C5["sqrt_s"], C5["m_lo"], C5["m_hi"], C5["m_z"], C5["gamma_z"], C5["sw2"], C5["alpha_em"],
                  C5["gev2_to_pb"]])
    return {f"mode{m}": extra_hadronic(vgx, pdf, vgx.DRELLYAN, np.concatenate([p, [float(m)]]), C5["seed"], n)
            for m in (0, 1)}


def extra_batch(vgx):
    """64 integrals, d 2..12, 1e4..1e7 samples, 10 iterations in one graph each."""
    import torch
    from synth import C3, batch_specs
    specs = batch_specs()
    ctxs = [vgx.vegas_create(s.kind, s.dim, C3["n_bins"], C3["alpha"], C3["seed"], s.stream, vgx.F32, s.params)
            for s in specs]
    try:
        t0 = time.perf_counter()
        b = vgx.batch_create(ctxs, [s.n for s in specs], 0, 0)
        t_create = time.perf_counter() - t0
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for it in range(C3["iterations"]):
                vgx.batch_iterate(b, it, len(specs))
            dt = time.perf_counter() - t0
            tile, block = vgx.batch_config(b)
        finally:
            vgx.batch_destroy(b)
        tot = sum(s.n for s in specs) * C3["iterations"]
        return {"events_per_s": tot / dt, "ms_per_iteration": dt / C3["iterations"] * 1e3,
                "events_per_iteration": tot // C3["iterations"], "autotuned_tile": tile, "autotuned_block": block,
                "create_and_autotune_ms": t_create * 1e3}
    finally:
        for c in ctxs:
            vgx.vegas_destroy(c)


def extra_members(vgx, grid):
    """Multi-member PDF evaluation: all 11 flavours of N_rep members at the
    2415 points of C7, FP64 outputs (kernel time from HIP events, median of
    5, and the wall time of one synchronous call)."""
    import torch
    from synth import C7, fk_points, synthetic_pdf_replicas
    x, q2 = fk_points(C7)
    xt, qt = torch.from_numpy(x).cuda(), torch.from_numpy(q2).cuda()
    members = synthetic_pdf_replicas(grid, max(C7["n_rep"]), C7["eps"], C7["seed"])
    out = {}
    for n_rep in C7["n_rep"]:
        ctx = vgx.pdf_create_set(grid.x_knots, grid.q2_knots, members[:n_rep])
        try:
            res = torch.empty((n_rep, 11, x.size), dtype=torch.float64, device="cuda")
            fn = lambda: vgx.pdf_interp_members(ctx, xt, qt, res)
            fn()
            ms = cuda_timed(fn)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            evals = n_rep * x.size * 11
            out[str(n_rep)] = {"kernel_ms": ms, "wall_ms": wall * 1e3, "flavour_evals_per_s": evals / (ms * 1e-3)}
        finally:
            vgx.pdf_destroy(ctx)
    return out


def extra_events(vgx):
    """Event generation: RAMBO (1e7 events, 4 particles, massless and massive),
    unweighting of the massive weights, and the LHE writer's rate on 2e5 kept
    events (formatting and writing by its thread, timed to the flush)."""
    import os
    import tempfile
    import torch
    n = 10_000_000
    out = {}
    w = torch.empty(n, dtype=torch.float64, device="cuda")
    mom = torch.empty((4, 4, n), dtype=torch.float64, device="cuda")
    for name, masses in (("rambo_massless_4", [0.0] * 4), ("rambo_massive_4", [173.0, 173.0, 4.7, 0.0])):
        fn = lambda: vgx.rambo_generate(masses, 1500.0, 21, 1, 0, 0, mom, w)
        fn()
        ms = cuda_timed(fn)
        byt = n * (4 * 4 + 1) * 8
        out[name] = {"events_per_s": n / (ms * 1e-3), "ms": ms, "written_GBps": byt / (ms * 1e-3) / 1e9,
                     "bytes_per_event": (4 * 4 + 1) * 8}
    idx = torch.empty(n, dtype=torch.int64, device="cuda")
    vgx.unweight(w, 21, 2, 99, idx)  # warm-up: the stream-ordered scratch pool
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for r in range(reps):
        k, wm = vgx.unweight(w, 21, 2, r, idx)
    dt = (time.perf_counter() - t0) / reps
    out["unweight_1e7"] = {"events_per_s": n / dt, "ms_including_sync": dt * 1e3, "kept": k,
                           "efficiency": k / n}
    m = 200_000
    with tempfile.TemporaryDirectory() as d:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with vgx.LheWriter(os.path.join(d, "ev.lhe")) as lw:
            lw.write(mom, None, m, [21, 21], [6, -6, 5, 21], [173.0, 173.0, 4.7, 0.0], 1500.0)
            t_queue = time.perf_counter() - t0
            lw.flush()
        dt = time.perf_counter() - t0
        size = os.path.getsize(os.path.join(d, "ev.lhe"))
    out["lhe_export_2e5"] = {"events_per_s": m / dt, "MB_per_s": size / dt / 1e6, "queue_call_ms": t_queue * 1e3}
    return out


def gpu_sums_on_oracle_sample(vgx, pdf, params, n_sample):
    """The GPU's S1, S2 over the same first n_sample events of iteration 0
    on the uniform grid (a fresh context: same seed, stream and counters)."""
    from synth import C2
    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], C2["seed"], 0, vgx.F32, params, pdf=pdf)
    try:
        r = vgx.vegas_iterate(v, n_sample, 0)
    finally:
        vgx.vegas_destroy(v)
    return r["s1"], r["s2"]


def compact_extras(vgx):
    """The other configurations, compactly: C0 (FP64 VEGAS on the d = 4
    Gaussian: its own size, time to 1e-4, and the chip-filling 1e9-sample
    roofline run), C1 (PDF interpolation, 1e8 queries), C3 (64 batched
    integrals) and C4 on the d = 8 narrow Gaussian (VEGAS vs flow)."""
    import numpy as np
    from synth import C0, C4
    out = {}
    g = extra_gauss(vgx)
    prm = np.concatenate([np.full(4, C0["centre"]), np.full(4, C0["sigma"])])
    # C0's own iteration size (1e5); the target needs ~4e7 samples
    tv = time_to_precision_vegas(vgx, None, prm, C0["n_per_iter"], kind=vgx.GAUSS, dim=4, seed=C0["seed"],
                                 max_iter=1500)
    out["c0_gauss4_f64"] = {"events_per_s_10x1e5": g["small"]["events_per_s"], "ms_10x1e5": g["small"]["ms_total"],
                            "time_to_1e-4": tv, "events_per_s_1e9": g["large"]["events_per_s"],
                            "kernel_ms_1e9": g["large"]["kernel_ms"],
                            "fp64_flops_per_sample": g["large"]["fp64_flops_per_sample"],
                            "frac_of_fp64_peak": g["large"]["frac_of_fp64_peak"]}
    pdfx = vgx.pdf_create(*_c1_grid_arrays())
    try:
        c1 = extra_pdf(vgx, pdfx)
    finally:
        vgx.pdf_destroy(pdfx)
    out["c1_pdf_interp_1e8"] = {k: {"queries_per_s": v["queries_per_s"], "frac_of_8TBps": v["frac_of_8TBps"],
                                    "ms": v["ms"]} for k, v in c1.items()}
    b = extra_batch(vgx)
    out["c3_batched_64"] = {"events_per_s": b["events_per_s"], "ms_per_iteration": b["ms_per_iteration"],
                            "autotuned_tile": b["autotuned_tile"], "autotuned_block": b["autotuned_block"]}
    d8 = C4["gauss_dim"]
    gp = np.concatenate([np.full(d8, C4["gauss_centre"]), np.full(d8, C4["gauss_sigma"])])
    # VEGAS: iterations of 1e7 (at most 30); flow: two warm-up iterations of
    # 1e6 (the narrow peak needs the second refinement before the flow's
    # training points see it), batches up to 1e7
    gv = time_to_precision_vegas(vgx, None, gp, 10_000_000, kind=vgx.GAUSS, dim=d8, seed=C4["seed"])
    gf = flow_pipeline(vgx, vgx.GAUSS, d8, gp, None, 1_000_000, warm_iters=2, steps=C4["steps"], batch=C4["batch"],
                       lr=C4["lr"], n_flow=10_000_000, seed=C4["seed"])
    keys = ("seconds", "seconds_excluding_training", "training_seconds", "reached", "rel_var_per_sample_flow",
            "rel_var_per_sample_vegas_refined_grid", "gain_trained_vs_identity_flow")
    out["c4_flow_gauss8"] = {"vegas_seconds": gv["seconds"], "vegas_reached": gv["reached"],
                             "flow": {k: gf.get(k) for k in keys}}
    return out


def _c1_grid_arrays():
    from synth import synthetic_pdf_grid
    g = synthetic_pdf_grid()
    return g.x_knots, g.q2_knots, g.xf


def main():
    args = parse()
    if args.copy_reference:
        copy_reference()
        return
    if args.pdf_only:
        pdf_only()
        return
    if args.extra:
        one_extra(args.extra, args.events)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    # the oracle's host legs first, before anything touches the GPU (its
    # worker processes are forks of this one)
    n_cpu = 4_000_000
    cpu = None if args.no_cpu else cpu_baseline(n_cpu)

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

    out_tail = {}
    # comparisons and the other configurations run before the headline's
    # warm-up and timed steps, which therefore run on a GPU whose clocks have
    # left idle
    if not args.no_flow:
        from synth import C4
        tv = time_to_precision_vegas(vgx, pdf, params, n)
        # one VEGAS warm-up iteration of 1e6 events: it refines the grid the
        # flow trains on (the training draws its own 1e5-point batches)
        tf = flow_pipeline(vgx, vgx.TTBAR, 3, params, pdf, 1_000_000, warm_iters=1, steps=C4["steps"],
                           batch=C4["batch"],
                           lr=C4["lr"], n_flow=n, seed=1000 + C2["seed"])
        out_tail["time_to_1e-4"] = {"vegas": tv, "flow": tf,
                                    "flow_faster_including_training": tf["seconds"] < tv["seconds"],
                                    "flow_faster_excluding_training": tf["seconds_excluding_training"] < tv["seconds"]}
    if not args.no_compact:
        out_tail["other_configs"] = compact_extras(vgx)
    if args.extras:
        out_tail["extras"] = {k: f() for k, f in extras_table(vgx, pdf, grid, params, n).items()}
    if cpu is not None:
        g1, g2 = gpu_sums_on_oracle_sample(vgx, pdf, params, n_cpu)
        out_tail["cpu_baseline"] = {
            "value": cpu["eps_1"], "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_cpu} events of iteration 0 (uniform grid), FP64 numpy, chunks of 250k: "
                      f"{cpu['secs_1']:.1f} s on one core; {cpu['secs_p']:.1f} s over {cpu['procs']} processes",
            "value_multi": cpu["eps_p"], "cores_multi": cpu["procs"],
            "oracle_s1": cpu["s1"], "oracle_s2": cpu["s2"], "gpu_s1": g1, "gpu_s2": g2,
            "gpu_vs_oracle_rel_s1": abs(g1 - cpu["s1"]) / abs(cpu["s1"]),
            "gpu_vs_oracle_rel_s2": abs(g2 - cpu["s2"]) / abs(cpu["s2"]),
        }

    v = vgx.vegas_create(vgx.TTBAR, 3, C2["n_bins"], C2["alpha"], C2["seed"], 0, vgx.F32, params, pdf=pdf)
    it = 0
    for _ in range(args.warmup):
        vgx.vegas_iterate(v, n, it)
        vgx.vegas_refine(v)
        it += 1
    torch.cuda.synchronize()
    # the kernel's own duration from HIP events around ten of the timed
    # launches, spread evenly (each event pair delays the next launch by a
    # few microseconds)
    vgx.vegas_set_timing(v, True, every=max(1, args.steps // 10))
    t0 = time.perf_counter()
    # GPU-resident loop: estimates, combination and refinement stay on the
    # device; the host reads the combined result once after the loop
    for _ in range(args.steps):
        vgx.vegas_iterate_async(v, n, it)
        vgx.vegas_refine(v)
        it += 1
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms, launches = vgx.vegas_kernel_time(v)
    vgx.vegas_set_timing(v, False)
    res = vgx.vegas_result(v)
    vgx.vegas_destroy(v)
    vgx.pdf_destroy(pdf)

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
            "traffic": measured_traffic(n),
            "traffic_unit": "bytes/launch (HBM, rocprofv3 FETCH_SIZE+WRITE_SIZE scaled by a 2 GiB copy)",
            "kernel": "k_vegas_iter<3,TTbar,PhiloxSrc<3>,true,false>",
            "kernel_avg_ms": kern_avg_s * 1e3,
            "flops_per_event": FLOPS_PER_EVENT_F32,
            "events_per_launch": n,
            "frac_per_flavour_count": FLOPS_PER_EVENT_PER_FLAVOUR_COUNT * n / kern_avg_s / PEAK_FP32,
            "flops_per_event_per_flavour_count": FLOPS_PER_EVENT_PER_FLAVOUR_COUNT,
        },
    }
    out.update(out_tail)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

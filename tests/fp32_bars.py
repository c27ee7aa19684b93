"""Per-event bars of the FP32 fused integrands against the FP64 oracle.

Error model.  The integrand is evaluated in FP32 (unit roundoff 2^-24 =
6e-8): the PDF lookup is a 16-term linear combination of node values with
Hermite weights (two of them negative), the luminosity a sum of positive
PDF products, the matrix element a closed form of a few dozen operations.
Where nothing cancels, each stage adds a few roundoffs, so the relative
error stays near 1e-6; the bar is 1e-5 per event, and the 99th percentile
must meet it too.  Where the PDFs are tiny (both x near 1, Hermite overshoot
next to the x = 1 knot) the stencil sums and the gg / q qbar luminosities
cancel, and the FP32 result carries eps32 times the magnitude of the
cancelling terms: a large relative error of a negligible weight.  Such
events may instead meet an absolute bar of 1e-7 of the mean weight, which
is looser than the relative bar only for weights below 1e-2 of the mean
(so every weight above that meets 1e-5 relative); how many events use it
depends on how many tiny weights the integrand has, so it is reported, not
bounded.  Events within 1e-6 (relative) of an x knot may be given the
neighbouring cell by the FP32 search; callers exclude and count them
(`keep`).
"""
import numpy as np

REL = 1e-5
FLOOR = 1e-7


def check_events(got, ref, keep, label=""):
    err = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = err / np.abs(ref)
    rel = np.where(err == 0.0, 0.0, rel)
    floor = FLOOR * np.mean(np.abs(ref))
    k = keep
    big = k & (np.abs(ref) >= 1e-3 * np.mean(np.abs(ref)))
    stats = (f"{label}: rel max {rel[k].max():.2e} p99 {np.percentile(rel[k], 99):.2e} "
             f"median {np.median(rel[k]):.2e}; weights >= 1e-3 of the mean: rel max {rel[big].max():.2e}; "
             f"over {REL:.0e}: {np.mean(rel[k] > REL):.2e} of {k.sum()} (excluded near knots: {(~keep).sum()})")
    print("  " + stats, flush=True)
    ok = (rel <= REL) | (err <= floor)
    assert ok[k].all(), stats + f"; worst beyond both bars {rel[k][~ok[k]].max():.2e}"
    assert np.percentile(rel[k], 99) <= REL, stats
    return rel

"""VEGAS adaptive importance sampling, FP64 (oracle) — test infrastructure.

Follows the thesis's Monte Carlo chapter:
  * estimator E_N = (1/N) sum f/p  (importance-sampling estimator equation);
  * its variance estimate, read as var(E_N) = ((1/N) sum w^2 - E_N^2)/(N-1)
    (the sample-variance equation equates a 1/(N-1) form with an 1/N form,
    which are not equal; this reading is the unbiased variance of the mean);
  * VEGAS (Sec. "Adaptive Monte Carlo: VEGAS algorithm"): separable grid with
    a fixed number of bins per dimension and adaptive widths; the per-
    iteration estimates are combined with inverse-variance weights and the
    chi^2/dof consistency check;
  * the sampling map is the inverse-transform method (Sec. "Inverse transform
    method") applied per dimension to the piecewise-constant density that
    the bin grid defines.

The refinement formula is not in the thesis (it cites Lepage 1978/1980 for
it).  Reading used, after Lepage: per dimension, accumulate d_i = sum of
(f J)^2 over the samples in bin i; smooth with a 3-point average of the
original values; normalise to p_i; damp with r_i = ((1 - p_i)/ln(1/p_i))^alpha;
re-bin so that each new bin holds an equal share of sum r, the old bins'
r being spread uniformly over their widths.

Sums use math.fsum (the exactly rounded sum), so they are exact up to one
final rounding, which is what the compensated GPU sums are compared with.

Pins: tests/test_oracle_vegas.py (closed-form Gaussian integrals, refinement
invariants, a hand-computed 3-bin rebin, map invariants, unbiasedness and
sigma-consistency over seeds).
"""
import math

import numpy as np

from .philox import sample_uniforms


def uniform_grid(dim, n_bins):
    """Edges e[j][k] = k / N."""
    return np.tile(np.arange(n_bins + 1, dtype=np.float64) / n_bins, (dim, 1))


def vegas_map(u, edges):
    """Map uniforms u (n, d) through the grid.

    i_j = min(floor(u_j N), N - 1), delta = u_j N - i_j,
    x_j = e_{j,i} + delta (e_{j,i+1} - e_{j,i}),  J = prod_j N (e_{j,i+1} - e_{j,i}).
    Returns x (n, d), J (n,), idx (n, d).
    """
    u = np.asarray(u, dtype=np.float64)
    n, d = u.shape
    nb = edges.shape[1] - 1
    t = u * nb
    idx = np.minimum(np.floor(t).astype(np.int64), nb - 1)
    delta = t - idx
    x = np.empty_like(u)
    jac = np.ones(n)
    for j in range(d):
        lo = edges[j, idx[:, j]]
        hi = edges[j, idx[:, j] + 1]
        width = hi - lo
        x[:, j] = lo + delta[:, j] * width
        jac = jac * (nb * width)
    return x, jac, idx


def iteration(f, edges, seed, stream, it, n, first=0):
    """One VEGAS iteration over sample indices first .. first+n-1.

    f maps x (n, d) -> values (n,).  Returns a dict with s1, s2, mean, var,
    hist (d, N) of (f J)^2 and the per-sample weights w.
    """
    d = edges.shape[0]
    nb = edges.shape[1] - 1
    idx = np.arange(first, first + n, dtype=np.uint64)
    u = sample_uniforms(seed, stream, it, idx, d)
    x, jac, bins = vegas_map(u, edges)
    w = f(x) * jac
    return estimate_from_weights(w, bins, d, nb)


def estimate_from_weights(w, bins, d, nb):
    n = w.shape[0]
    w2 = w * w
    s1 = math.fsum(w)
    s2 = math.fsum(w2)
    hist = np.zeros((d, nb))
    for j in range(d):
        order = np.argsort(bins[:, j], kind="stable")
        b_sorted = bins[order, j]
        w_sorted = w2[order]
        cuts = np.searchsorted(b_sorted, np.arange(nb + 1))
        for i in range(nb):
            hist[j, i] = math.fsum(w_sorted[cuts[i]:cuts[i + 1]])
    mean, var = mean_var(s1, s2, n)
    return dict(s1=s1, s2=s2, n=n, mean=mean, var=var, hist=hist, w=w)


def mean_var(s1, s2, n):
    """E = S1/n, var(E) = max(S2/n - E^2, 0)/(n - 1)."""
    mean = s1 / n
    var = max(s2 / n - mean * mean, 0.0) / (n - 1) if n > 1 else 0.0
    return mean, var


def refine(edges, hist, alpha):
    """Return the refined edges (Lepage's smoothing, damping and re-binning)."""
    d, nb1 = edges.shape
    nb = nb1 - 1
    out = edges.copy()
    for j in range(d):
        dj = [float(v) for v in hist[j]]
        # an all-zero histogram, or one holding a non-finite weight (an
        # iteration the combination excludes), leaves the dimension unchanged
        if not all(math.isfinite(v) for v in dj) or math.fsum(dj) <= 0.0:
            continue
        sm = [0.0] * nb
        if nb == 1:
            sm[0] = dj[0]
        else:
            sm[0] = (dj[0] + dj[1]) / 2.0
            for i in range(1, nb - 1):
                sm[i] = (dj[i - 1] + dj[i] + dj[i + 1]) / 3.0
            sm[nb - 1] = (dj[nb - 2] + dj[nb - 1]) / 2.0
        tot = math.fsum(sm)
        r = []
        for i in range(nb):
            p = sm[i] / tot
            if p <= 0.0:
                r.append(0.0)
            elif p >= 1.0:
                r.append(1.0)
            else:
                r.append(((1.0 - p) / math.log(1.0 / p)) ** alpha)
        out[j] = rebin(edges[j], r)
    return out


def rebin(e, r):
    """New edges with equal shares R/N of sum(r) per new bin, where r_i is
    spread uniformly over old bin i."""
    nb = len(r)
    R = math.fsum(r)
    new = np.empty(nb + 1)
    new[0] = e[0]
    new[nb] = e[nb]
    target_step = R / nb
    i = 0
    acc = 0.0  # sum of r over old bins < i
    for k in range(1, nb):
        target = k * target_step
        while i < nb - 1 and acc + r[i] < target:
            acc += r[i]
            i += 1
        if r[i] > 0.0:
            frac = (target - acc) / r[i]
            frac = min(max(frac, 0.0), 1.0)
        else:
            frac = 0.0
        new[k] = e[i] + frac * (e[i + 1] - e[i])
    return new


def combine(means, variances):
    """Inverse-variance combination and chi^2/dof (VEGAS check equation).

    E_bar = S^2 sum E_i/S_i^2, 1/S^2 = sum 1/S_i^2,
    chi^2/dof = 1/(M-1) sum (E_i - E_bar)^2 / S_i^2.
    If some S_i^2 is zero, that estimate is exact: return it with sigma 0.
    """
    means = [float(m) for m in means]
    variances = [float(v) for v in variances]
    for m, v in zip(means, variances):
        if v == 0.0:
            return m, 0.0, 0.0
    wsum = math.fsum(1.0 / v for v in variances)
    ebar = math.fsum(m / v for m, v in zip(means, variances)) / wsum
    sigma = math.sqrt(1.0 / wsum)
    M = len(means)
    chi2 = math.fsum((m - ebar) ** 2 / v for m, v in zip(means, variances)) / (M - 1) if M > 1 else 0.0
    return ebar, sigma, chi2


def run(f, dim, n_bins, alpha, iterations, n, seed, stream=0, edges=None):
    """Full VEGAS run: every iteration refines and all are combined."""
    if edges is None:
        edges = uniform_grid(dim, n_bins)
    res = []
    for it in range(iterations):
        r = iteration(f, edges, seed, stream, it, n)
        res.append(r)
        edges = refine(edges, r["hist"], alpha)
    ebar, sigma, chi2 = combine([r["mean"] for r in res], [r["var"] for r in res])
    return dict(mean=ebar, sigma=sigma, chi2_dof=chi2, iterations=res, edges=edges)

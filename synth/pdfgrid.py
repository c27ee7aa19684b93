"""Synthetic PDF grid in the LHAPDF layout (knots in x and Q^2, subgrids).

The grid imitates the shape of a real NLO set: 196 log-spaced x knots in
[1e-9, 1] and three Q subgrids split at the charm and bottom thresholds, the
threshold knot duplicated in both neighbours (the thesis's PDF grid section
describes subgrids split at quark-mass thresholds; the knot ranges are those
of the NNPDF3.1 example it quotes).  Node values follow

    xf(x, Q^2) = A x^a (1 - x)^b (1 + c sqrt(x)),
    L = ln( ln(Q^2/Lambda^2) / ln(Q0^2/Lambda^2) ),
    a = a0 - 0.08 L,  b = b0 + 0.5 L,  A = A0 (1 + 0.1 L),

with seeded per-flavour (a0, b0, c) and A0 chosen so that the momentum sum
rule  sum_f int_0^1 xf dx = 1  holds exactly at Q0 for the *continuous*
functions (Beta-function integrals).  Charm is zero below 1.3 GeV and
bottom below 4.75 GeV, which is what makes the subgrid split matter.

Only inputs are produced here; nothing in this file interpolates.
"""
from dataclasses import dataclass

import numpy as np
from scipy.special import beta as beta_fn

from .configs import C1, FLAVOURS

# Momentum fraction carried by each flavour at Q0 (sums to 1 over the
# flavours present at Q0).  Heavy flavours get a nominal fraction that only
# sets their normalisation above threshold.
_MOMENTUM_FRACTION = {
    21: 0.45, 2: 0.27, 1: 0.14, -2: 0.04, -1: 0.05, 3: 0.025, -3: 0.025,
    4: 0.010, -4: 0.010, 5: 0.005, -5: 0.005,
}
_LIGHT_AT_Q0 = (21, 2, 1, -2, -1, 3, -3)


@dataclass
class PdfGridData:
    """Knots and node values of a PDF grid.

    x_knots : (n_x,) ascending, shared by all subgrids.
    q2_knots: list of (n_q[s],) ascending arrays, one per subgrid; the last
              knot of subgrid s equals the first knot of subgrid s+1.
    xf      : list of (n_flav, n_q[s], n_x) arrays of x*f node values.
    params  : per-flavour (A0, a0, b0, c) used to build the values.
    """
    x_knots: np.ndarray
    q2_knots: list
    xf: list
    params: dict
    lambda_qcd: float
    q0: float

    @property
    def n_flav(self):
        return self.xf[0].shape[0]

    def xf_exact(self, flav_index, x, q2):
        """The continuous function the nodes were sampled from (subgrid rule
        for the heavy-flavour cut-offs included).  Used as an input-level
        check only."""
        pid = FLAVOURS[flav_index]
        A0, a0, b0, c = self.params[pid]
        x = np.asarray(x, dtype=np.float64)
        q2 = np.asarray(q2, dtype=np.float64)
        lam2 = self.lambda_qcd ** 2
        L = np.log(np.log(q2 / lam2) / np.log(self.q0 ** 2 / lam2))
        a = a0 - 0.08 * L
        b = b0 + 0.5 * L
        A = A0 * (1.0 + 0.1 * L)
        val = A * x ** a * (1.0 - x) ** b * (1.0 + c * np.sqrt(x))
        return val


def _flavour_params(rng):
    params = {}
    for pid in FLAVOURS:
        if pid == 21:
            a0, b0, c = -0.1, 5.0, 0.0
        elif pid in (1, 2):  # valence-like
            a0 = 0.5 + rng.uniform(-0.05, 0.05)
            b0 = 3.0 + rng.uniform(-0.3, 0.3)
            c = rng.uniform(0.0, 1.0)
        else:  # sea-like
            a0 = -0.15 + rng.uniform(-0.03, 0.03)
            b0 = 7.0 + rng.uniform(-0.5, 0.5)
            c = rng.uniform(-0.5, 0.5)
        # The stored quantity is x f = A x^a (1-x)^b (1 + c sqrt x), so the
        # momentum integral int_0^1 x f dx = A [B(a+1,b+1) + c B(a+1.5,b+1)].
        norm = beta_fn(a0 + 1.0, b0 + 1.0) + c * beta_fn(a0 + 1.5, b0 + 1.0)
        A0 = _MOMENTUM_FRACTION[pid] / norm
        params[pid] = (float(A0), float(a0), float(b0), float(c))
    return params


def synthetic_pdf_grid(cfg=C1):
    """Build the synthetic grid of configuration C1 (seeded)."""
    rng = np.random.default_rng(cfg["grid_seed"])
    n_x = cfg["n_x"]
    lx = np.log10(cfg["x_min"]) + (np.log10(cfg["x_max"]) - np.log10(cfg["x_min"])) * np.arange(n_x) / (n_x - 1)
    x_knots = 10.0 ** lx
    x_knots[0] = cfg["x_min"]
    x_knots[-1] = cfg["x_max"]

    q_edges = cfg["q_edges"]
    q2_knots = []
    for s, nq in enumerate(cfg["nq_per_sub"]):
        lo, hi = q_edges[s] ** 2, q_edges[s + 1] ** 2
        k = np.exp(np.linspace(np.log(lo), np.log(hi), nq))
        k[0], k[-1] = lo, hi
        q2_knots.append(k)

    params = _flavour_params(rng)
    grid = PdfGridData(x_knots=x_knots, q2_knots=q2_knots, xf=[], params=params,
                       lambda_qcd=cfg["lambda_qcd"], q0=cfg["q0"])
    X = x_knots[None, :]
    for s, q2 in enumerate(q2_knots):
        vals = np.zeros((len(FLAVOURS), len(q2), n_x))
        for fi, pid in enumerate(FLAVOURS):
            if abs(pid) == 4 and s < 1:
                continue
            if abs(pid) == 5 and s < 2:
                continue
            vals[fi] = grid.xf_exact(fi, X, q2[:, None])
        grid.xf.append(vals)
    return grid


def _perturb_interior(knots, frac, rng):
    """Knots moved, in the logarithm, by up to +-frac of the local spacing;
    the two end knots stay (they are the grid limits or subgrid thresholds)."""
    lk = np.log(knots)
    h = np.diff(lk)
    out = lk.copy()
    for k in range(1, len(lk) - 1):
        out[k] = lk[k] + frac * min(h[k - 1], h[k]) * rng.uniform(-1.0, 1.0)
    res = np.exp(out)
    res[0], res[-1] = knots[0], knots[-1]
    assert np.all(np.diff(res) > 0)
    return res


def nonuniform_pdf_grid(cfg=C1, frac=0.2, seed=11):
    """The grid of `synthetic_pdf_grid` on knots that are not evenly spaced:
    every interior x knot and every interior Q^2 knot of each subgrid moved
    by up to +-frac of a spacing in the logarithm (seeded), the same
    continuous functions sampled at the moved knots.  Real PDF sets are not
    evenly spaced in ln x or ln Q^2; this exercises the general cell search
    and the uneven-spacing slope ratios of an interpolator."""
    base = synthetic_pdf_grid(cfg)
    rng = np.random.default_rng(seed)
    x_knots = _perturb_interior(base.x_knots, frac, rng)
    q2_knots = [_perturb_interior(q, frac, rng) for q in base.q2_knots]
    grid = PdfGridData(x_knots=x_knots, q2_knots=q2_knots, xf=[], params=base.params,
                       lambda_qcd=base.lambda_qcd, q0=base.q0)
    X = x_knots[None, :]
    for s, q2 in enumerate(q2_knots):
        vals = np.zeros((len(FLAVOURS), len(q2), len(x_knots)))
        for fi, pid in enumerate(FLAVOURS):
            if abs(pid) == 4 and s < 1:
                continue
            if abs(pid) == 5 and s < 2:
                continue
            vals[fi] = grid.xf_exact(fi, X, q2[:, None])
        grid.xf.append(vals)
    return grid


def momentum_sum_at_q0(grid):
    """Exact momentum sum of the continuous functions at Q0 (should be 1)."""
    tot = 0.0
    for pid in _LIGHT_AT_Q0:
        A0, a0, b0, c = grid.params[pid]
        tot += A0 * (beta_fn(a0 + 1.0, b0 + 1.0) + c * beta_fn(a0 + 1.5, b0 + 1.0))
    return tot


def synthetic_pdf_replicas(grid, n_rep, eps, seed):
    """n_rep members (lists of per-subgrid (n_flav, n_q, n_x) arrays) around
    `grid`: member m = grid times 1 + eps (a + b ln x / ln 1e-9), with (a, b)
    standard normal per member and flavour, shared by all subgrids."""
    rng = np.random.default_rng(seed)
    L = np.log(grid.x_knots) / np.log(1e-9)
    members = []
    for _ in range(n_rep):
        ab = rng.standard_normal((len(FLAVOURS), 2))
        fac = 1.0 + eps * (ab[:, 0:1] + ab[:, 1:2] * L[None, :])  # (n_flav, n_x)
        members.append([v * fac[:, None, :] for v in grid.xf])
    return members

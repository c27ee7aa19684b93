"""PDF and alpha_s values outside the grid (oracle) — test infrastructure.

Thesis, PDF chapter (the LHAPDF paragraphs on extrapolation and the alpha_s
paragraph).  Three behaviours outside the grid's (x, Q^2) box:

  ERROR    no value (NaN): the "raise an error" option.
  FREEZE   the value at the nearest point of the grid: x and Q^2 clamped to
           the grid's ranges, then interpolated.
  CONTINUE the legacy continuation (the default the thesis describes):
    low x (x < x_0, Q^2 inside): a straight line in ln x through the values
      at the two lowest x knots (x_0, x_1) at that Q^2, drawn through ln xf
      when both values exceed 1e-3, else through xf itself;
    high Q^2 (Q^2 > Q^2_max): the same rule in ln Q^2, through the values on
      the two highest Q^2 knots;
    low Q^2 (Q^2 < Q^2_min): xf = G0 r^((gamma - 1) r + 1), r = Q^2/Q^2_min,
      G0 = xf(x, Q^2_min), gamma the anomalous dimension at Q^2_min; this
      tends to G0 r^gamma as r -> 1 and to G0 r as r -> 0;
    x and Q^2 both outside: the x rule first, on the Q^2 rows the Q^2 rule
      reads, then the Q^2 rule.
  x above the top knot has no continuation (NaN in ERROR and CONTINUE).

Readings (the passage is garbled or silent):
  * gamma = d ln xf / d ln Q^2.  The printed derivative with respect to Q^2
    would make the exponent carry dimensions, and the stated limits need the
    logarithmic derivative.
  * gamma is the logarithmic derivative at Q^2_min of what the grid gives
    just above Q^2_min at this x, so that ln xf and its derivative in ln Q^2
    are continuous across Q^2_min.  For x_0 <= x the lowest Q^2 cell of the
    lowest subgrid is interpolated bilinearly: with G0, G1 the values on its
    two rows at x (linear in ln x between the bracketing knots),
    gamma = (G1 - G0) / (db G0), db = ln Q^2_1 - ln Q^2_0.  For x < x_0 the
    grid gives the low-x line through the cell's columns at x_0 and x_1,
    whose values f_k (row 0) move with slopes f'_k = (row 1 - row 0)/db; at
    the line's fraction s, gamma = (1-s) f'_0/f_0 + s f'_1/f_1 on the log
    branch and ((1-s) f'_0 + s f'_1) / G0 on the linear one.  G0 = 0 gives
    xf = 0.
  * The high-Q^2 rows are the top subgrid's last two, the low-Q^2 rows the
    lowest subgrid's first two, each read at x with the rule of its edge cell
    (linear in ln x); a threshold knot never switches subgrid here.
  * alpha_s: alpha_s(Q^2_max) above the top knot in every mode; below the
    lowest knot NaN (ERROR), alpha_s(Q^2_min) (FREEZE), or the low-x straight
    line rule in ln Q^2 through the two lowest knots (CONTINUE: the text's
    logarithmic-gradient continuation "similar to the low-x behaviour"; its
    "Q > Q_min" is read as Q < Q_min).
  * Non-positive or non-finite x or Q^2: NaN in every mode.

Pins: tests/test_oracle_pdf_extrap.py -- in-grid values unchanged; freeze
constant along the outward directions; exact continuation of power laws in x
and Q^2 (log branch) and of functions linear in ln x (linear branch), corners
included; a hand-computed low-Q^2 value; continuity of xf and of
d ln xf / d ln Q^2 across Q^2_min (with an independent finite difference of
the in-grid interpolant); the Q^2 -> 0 limit; continuity across x_0 at low
Q^2; alpha_s power laws continued exactly.
"""
import math

import numpy as np

from . import alphas as _alphas
from . import pdf as _pdf

ERROR, FREEZE, CONTINUE = 0, 1, 2
POSITIVE = 1e-3


def continue_line(t, y0, y1):
    """Value at fraction t (any real number) of the straight line through
    (0, y0) and (1, y1), drawn through ln y where both values exceed 1e-3
    and through y otherwise; elementwise."""
    y0 = np.asarray(y0, dtype=np.float64)
    y1 = np.asarray(y1, dtype=np.float64)
    pos = (y0 > POSITIVE) & (y1 > POSITIVE)
    l0 = np.log(np.where(pos, y0, 1.0))
    l1 = np.log(np.where(pos, y1, 1.0))
    return np.where(pos, np.exp(l0 + t * (l1 - l0)), y0 + t * (y1 - y0))


def row_values(grid, s, k, x):
    """xf of every flavour on Q^2 row k of subgrid s at x <= x_max: linear in
    ln x between the bracketing x knots, continued in x below x_0."""
    xk = grid.x_knots
    ax = np.log(xk)
    F = grid.xf[s][:, k, :]
    a = math.log(x)
    if x < xk[0]:
        return continue_line((a - ax[0]) / (ax[1] - ax[0]), F[:, 0], F[:, 1])
    i = min(int(np.searchsorted(xk, x, side="right")) - 1, len(xk) - 2)
    t = (a - ax[i]) / (ax[i + 1] - ax[i])
    return F[:, i] + t * (F[:, i + 1] - F[:, i])


def _low_x(grid, x, q2):
    xk = grid.x_knots
    f0 = _pdf.interp(grid, xk[0], q2)[:, 0]
    f1 = _pdf.interp(grid, xk[1], q2)[:, 0]
    t = (math.log(x) - math.log(xk[0])) / (math.log(xk[1]) - math.log(xk[0]))
    return continue_line(t, f0, f1)


def _high_q(grid, x, q2):
    s = len(grid.q2_knots) - 1
    qk = grid.q2_knots[s]
    n = len(qk)
    g0 = row_values(grid, s, n - 2, x)
    g1 = row_values(grid, s, n - 1, x)
    t = (math.log(q2) - math.log(qk[n - 2])) / (math.log(qk[n - 1]) - math.log(qk[n - 2]))
    return continue_line(t, g0, g1)


def anomalous_dimension(grid, x):
    """gamma = d ln xf / d ln Q^2 at Q^2_min, taken from just above it (per
    flavour; not finite where G0 = 0)."""
    qk = grid.q2_knots[0]
    db = math.log(qk[1]) - math.log(qk[0])
    xk = grid.x_knots
    with np.errstate(divide="ignore", invalid="ignore"):
        if x >= xk[0]:
            g0 = row_values(grid, 0, 0, x)
            g1 = row_values(grid, 0, 1, x)
            return (g1 - g0) / (db * g0)
        lo, hi = grid.xf[0][:, 0, :], grid.xf[0][:, 1, :]
        f0, f1 = lo[:, 0], lo[:, 1]
        d0, d1 = (hi[:, 0] - lo[:, 0]) / db, (hi[:, 1] - lo[:, 1]) / db
        s = (math.log(x) - math.log(xk[0])) / (math.log(xk[1]) - math.log(xk[0]))
        pos = (f0 > POSITIVE) & (f1 > POSITIVE)
        g0 = continue_line(s, f0, f1)
        return np.where(pos, (1.0 - s) * d0 / f0 + s * d1 / f1, ((1.0 - s) * d0 + s * d1) / g0)


def _low_q(grid, x, q2):
    qk = grid.q2_knots[0]
    g0 = row_values(grid, 0, 0, x)
    gamma = anomalous_dimension(grid, x)
    r = q2 / qk[0]
    lr = math.log(q2) - math.log(qk[0])
    out = np.zeros_like(g0)
    nz = g0 != 0.0
    out[nz] = g0[nz] * np.exp(((gamma[nz] - 1.0) * r + 1.0) * lr)
    return out


def interp_extrap(grid, x, q2, mode):
    """xf of every flavour (n_flav, n) at (x, q2) with the given behaviour
    outside the grid; in-grid queries are the interpolator's values."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    q2 = np.atleast_1d(np.asarray(q2, dtype=np.float64))
    out = _pdf.interp(grid, x, q2)
    if mode == ERROR:
        return out
    xk = grid.x_knots
    q2min, q2max = grid.q2_knots[0][0], grid.q2_knots[-1][-1]
    for n in range(x.shape[0]):
        xi, qi = float(x[n]), float(q2[n])
        if not (math.isfinite(xi) and math.isfinite(qi) and xi > 0.0 and qi > 0.0):
            continue
        in_x = xk[0] <= xi <= xk[-1]
        in_q = q2min <= qi <= q2max
        if in_x and in_q:
            continue
        if mode == FREEZE:
            xc = min(max(xi, xk[0]), xk[-1])
            qc = min(max(qi, q2min), q2max)
            out[:, n] = _pdf.interp(grid, xc, qc)[:, 0]
        elif xi <= xk[-1]:
            if in_q:
                out[:, n] = _low_x(grid, xi, qi)
            elif qi > q2max:
                out[:, n] = _high_q(grid, xi, qi)
            else:
                out[:, n] = _low_q(grid, xi, qi)
    return out


def alphas_extrap(table, q2, mode):
    """alpha_s at q2 (n,) with the given behaviour below the lowest knot."""
    q2 = np.atleast_1d(np.asarray(q2, dtype=np.float64))
    out = _alphas.interp(table, q2)
    ok = np.isfinite(q2) & (q2 > 0.0)
    out[~ok] = np.nan
    below = ok & (q2 < table.q2_knots[0][0])
    if mode == FREEZE:
        out[below] = table.values[0][0]
    elif mode == CONTINUE and below.any():
        qk, v = table.q2_knots[0], table.values[0]
        t = (np.log(q2[below]) - math.log(qk[0])) / (math.log(qk[1]) - math.log(qk[0]))
        out[below] = continue_line(t, v[0], v[1])
    return out

"""Log-cubic interpolation of alpha_s(Q) (oracle) — test infrastructure.

Thesis, PDF chapter (alpha_s paragraphs, LHAPDF and PDFFlow): PDF sets carry
alpha_s at knots on the log Q line; the interpolation is a cubic Hermite
spline, with the improved treatment of subgrids split at flavour thresholds,
and a constant value alpha_s(Q_max) above the top knot.  The text's rule for
the region below the lowest knot is garbled (it writes "Q > Q_min" where the
context needs Q < Q_min); that region is read as out of range (NaN), as for
the PDFs' "raise an error" mode.

Definition implemented: b = ln Q^2 (the Hermite rule with secant-average
slopes is invariant under the affine change ln Q -> ln Q^2); subgrid s with
Q2lo(s) <= Q^2 < Q2hi(s), the upper subgrid winning at thresholds and the
last one closed at its top; cell j with b_j <= b < b_{j+1}; if
1 <= j <= n_q - 3 the cubic Hermite between knots j and j+1 with node slopes
the average of the two adjacent secants, else linear on the cell.

Pins: tests/test_oracle_alphas.py -- node values exact, quadratics in b
reproduced on the uniformly spaced subgrids, linear functions everywhere,
constant continuation above the top, NaN below the bottom, and the one-loop
function the synthetic table samples within the interpolation error.
"""
import numpy as np

from .pdf import find_cell, find_subgrid, hermite


def interp(table, q2):
    """alpha_s at q2 (n,) from an alpha_s table (knots/values per subgrid)."""
    q2 = np.atleast_1d(np.asarray(q2, dtype=np.float64))
    out = np.full(q2.shape, np.nan)
    top = table.q2_knots[-1][-1]
    above = q2 > top
    out[above] = table.values[-1][-1]
    sub = find_subgrid(table.q2_knots, q2)
    b = np.log(np.where(q2 > 0, q2, 1.0))
    for s in range(len(table.q2_knots)):
        sel = np.nonzero(sub == s)[0]
        if sel.size == 0:
            continue
        bq = np.log(table.q2_knots[s])
        v = table.values[s]
        nq = len(bq)
        j = find_cell(table.q2_knots[s], q2[sel])
        cubic = (j >= 1) & (j <= nq - 3)
        lin = sel[~cubic]
        if lin.size:
            jl = j[~cubic]
            t = (b[lin] - bq[jl]) / (bq[jl + 1] - bq[jl])
            out[lin] = v[jl] + t * (v[jl + 1] - v[jl])
        cub = sel[cubic]
        if cub.size:
            jc = j[cubic]
            db = bq[jc + 1] - bq[jc]
            t = (b[cub] - bq[jc]) / db
            m0 = 0.5 * ((v[jc + 1] - v[jc]) / db + (v[jc] - v[jc - 1]) / (bq[jc] - bq[jc - 1]))
            m1 = 0.5 * ((v[jc + 2] - v[jc + 1]) / (bq[jc + 2] - bq[jc + 1]) + (v[jc + 1] - v[jc]) / db)
            out[cub] = hermite(v[jc], v[jc + 1], m0 * db, m1 * db, t)
    return out

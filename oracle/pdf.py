"""Log-bicubic PDF interpolation on subgrids (oracle) — test infrastructure.

Follows the thesis's description of LHAPDF6 interpolation (Sec. "Parton
Distribution Functions", LHAPDF paragraphs) and PDFFlow's Subgrid design:
values xf on knots in (x, Q^2), possibly split into subgrids at quark-mass
thresholds; interpolation by cubic Hermite splines in (ln x, ln Q^2) on the
4 neighbouring knots per axis; bilinear interpolation where the 4-knot
stencil is not available.

Definition implemented (readings where the thesis is silent):
  a = ln x, b = ln Q^2.
  Subgrid s: the one with Q2lo(s) <= Q^2 < Q2hi(s); the last subgrid is
  closed at its top; at a threshold the upper subgrid wins.
  Cell i: x_i <= x < x_{i+1} (i = n_x - 2 at x = x_max); cell j likewise in
  the subgrid's Q^2 knots.
  If 1 <= i <= n_x - 3 and 1 <= j <= n_q(s) - 3: bicubic --
     for each of the 4 rows r = j-1..j+2, a cubic Hermite in a between
     knots i and i+1, with node slopes m_k the average of the two adjacent
     secants (LHAPDF6's rule, Buckley et al. 2015 -- the thesis cites that
     paper but does not print the rule);
     then a cubic Hermite in b through the 4 row values, same slope rule.
  Otherwise: bilinear in (a, b) on the 4 cell corners.
  H(v0, v1, d0, d1, t) = (2t^3-3t^2+1) v0 + (t^3-2t^2+t) d0
                       + (-2t^3+3t^2) v1 + (t^3-t^2) d1,
  where d0, d1 are slopes times the cell width.
  Out-of-grid queries give NaN ("raise an error" extrapolation mode).

Pins: tests/test_oracle_pdf.py -- node values exact; quadratics in (a, b)
reproduced on uniformly spaced subgrids; linear functions on non-uniform
spacing; bilinear zones reproduce bilinear functions; the Hermite kernel
with exact derivatives reproduces cubics (so the tensor product reproduces
bicubics); C^1 continuity across interior cells; the momentum sum rule of
the synthetic grid up to interpolation error; a brute-force scalar
evaluation on a tiny grid.
"""
import numpy as np


def hermite(v0, v1, d0, d1, t):
    t2 = t * t
    t3 = t2 * t
    return ((2 * t3 - 3 * t2 + 1) * v0 + (t3 - 2 * t2 + t) * d0
            + (-2 * t3 + 3 * t2) * v1 + (t3 - t2) * d1)


def find_subgrid(q2_knots, q2):
    """Index of the subgrid holding q2 (upper one at thresholds), -1 if out."""
    q2 = np.asarray(q2, dtype=np.float64)
    s = np.full(q2.shape, -1, dtype=np.int64)
    n_sub = len(q2_knots)
    for k in range(n_sub):
        lo, hi = q2_knots[k][0], q2_knots[k][-1]
        if k == n_sub - 1:
            inside = (q2 >= lo) & (q2 <= hi)
        else:
            inside = (q2 >= lo) & (q2 < hi)
        s = np.where(inside, k, s)  # later (upper) subgrids overwrite
    return s


def find_cell(knots, v):
    """i with knots[i] <= v < knots[i+1]; n-2 at the top knot."""
    i = np.searchsorted(knots, v, side="right") - 1
    return np.clip(i, 0, len(knots) - 2)


def interp(grid, x, q2):
    """xf for every flavour at (x, q2): returns (n_flav, n) FP64."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    q2 = np.atleast_1d(np.asarray(q2, dtype=np.float64))
    n = x.shape[0]
    xk = grid.x_knots
    nx = len(xk)
    nf = grid.n_flav
    out = np.full((nf, n), np.nan)
    ax = np.log(xk)
    sub = find_subgrid(grid.q2_knots, q2)
    in_x = (x >= xk[0]) & (x <= xk[-1])
    a = np.log(x)
    b = np.log(q2)
    for s in range(len(grid.q2_knots)):
        sel = np.nonzero((sub == s) & in_x)[0]
        if sel.size == 0:
            continue
        qk = grid.q2_knots[s]
        bq = np.log(qk)
        nq = len(qk)
        F = grid.xf[s]  # (nf, nq, nx)
        i = find_cell(xk, x[sel])
        j = find_cell(qk, q2[sel])
        cubic = (i >= 1) & (i <= nx - 3) & (j >= 1) & (j <= nq - 3)
        # bilinear part
        lin = sel[~cubic]
        if lin.size:
            il, jl = i[~cubic], j[~cubic]
            ta = (a[lin] - ax[il]) / (ax[il + 1] - ax[il])
            tb = (b[lin] - bq[jl]) / (bq[jl + 1] - bq[jl])
            f00 = F[:, jl, il]
            f01 = F[:, jl, il + 1]
            f10 = F[:, jl + 1, il]
            f11 = F[:, jl + 1, il + 1]
            lo = f00 + ta * (f01 - f00)
            hi = f10 + ta * (f11 - f10)
            out[:, lin] = lo + tb * (hi - lo)
        cub = sel[cubic]
        if cub.size:
            ic, jc = i[cubic], j[cubic]
            da = ax[ic + 1] - ax[ic]
            ta = (a[cub] - ax[ic]) / da
            rows = []
            for r in range(4):
                jr = jc - 1 + r
                fm = F[:, jr, ic - 1]
                f0 = F[:, jr, ic]
                f1 = F[:, jr, ic + 1]
                f2 = F[:, jr, ic + 2]
                m0 = 0.5 * ((f1 - f0) / da + (f0 - fm) / (ax[ic] - ax[ic - 1]))
                m1 = 0.5 * ((f2 - f1) / (ax[ic + 2] - ax[ic + 1]) + (f1 - f0) / da)
                rows.append(hermite(f0, f1, m0 * da, m1 * da, ta))
            db = bq[jc + 1] - bq[jc]
            tb = (b[cub] - bq[jc]) / db
            vm, v0, v1, v2 = rows
            m0 = 0.5 * ((v1 - v0) / db + (v0 - vm) / (bq[jc] - bq[jc - 1]))
            m1 = 0.5 * ((v2 - v1) / (bq[jc + 2] - bq[jc + 1]) + (v1 - v0) / db)
            out[:, cub] = hermite(v0, v1, m0 * db, m1 * db, tb)
    return out


def interp_scalar(grid, flav, x, q2):
    """Brute-force scalar evaluation (pure Python), for tiny-grid pins."""
    import math
    xk = [float(v) for v in grid.x_knots]
    nx = len(xk)
    sub = -1
    for k, qk in enumerate(grid.q2_knots):
        lo, hi = float(qk[0]), float(qk[-1])
        last = k == len(grid.q2_knots) - 1
        if lo <= q2 and (q2 < hi or (last and q2 <= hi)):
            sub = k
    if sub < 0 or not (xk[0] <= x <= xk[-1]):
        return float("nan")
    qk = [float(v) for v in grid.q2_knots[sub]]
    nq = len(qk)
    i = max(k for k in range(nx - 1) if xk[k] <= x)
    j = max(k for k in range(nq - 1) if qk[k] <= q2)
    F = grid.xf[sub][flav]
    A = [math.log(v) for v in xk]
    B = [math.log(v) for v in qk]
    a, b = math.log(x), math.log(q2)
    if 1 <= i <= nx - 3 and 1 <= j <= nq - 3:
        def herm_axis(vals, knots, k, t):
            h = knots[k + 1] - knots[k]
            s0 = 0.5 * ((vals[k + 1] - vals[k]) / h + (vals[k] - vals[k - 1]) / (knots[k] - knots[k - 1]))
            s1 = 0.5 * ((vals[k + 2] - vals[k + 1]) / (knots[k + 2] - knots[k + 1]) + (vals[k + 1] - vals[k]) / h)
            return hermite(vals[k], vals[k + 1], s0 * h, s1 * h, t)
        ta = (a - A[i]) / (A[i + 1] - A[i])
        col = {}
        for r in range(j - 1, j + 3):
            col[r] = herm_axis([float(v) for v in F[r]], A, i, ta)
        tb = (b - B[j]) / (B[j + 1] - B[j])
        vals = [0.0] * nq
        for r in range(j - 1, j + 3):
            vals[r] = col[r]
        return herm_axis(vals, B, j, tb)
    ta = (a - A[i]) / (A[i + 1] - A[i])
    tb = (b - B[j]) / (B[j + 1] - B[j])
    lo = F[j][i] + ta * (F[j][i + 1] - F[j][i])
    hi = F[j + 1][i] + ta * (F[j + 1][i + 1] - F[j + 1][i])
    return float(lo + tb * (hi - lo))

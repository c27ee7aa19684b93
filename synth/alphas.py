"""Synthetic alpha_s(Q) table on the Q^2 knots of the synthetic PDF grid.

PDF sets carry alpha_s at a list of Q values (the thesis's alpha_s paragraphs
of the PDF chapter); this one is one-loop running with 5 active flavours
above the bottom threshold, matched continuously to 4 and 3 flavours below
the bottom and charm thresholds:
    1/alpha(Q^2) = 1/alpha(Q_ref^2) + b0(nf) ln(Q^2/Q_ref^2),  b0 = (33 - 2 nf)/(12 pi),
anchored at alpha(M_Z) = 0.118.  The knots are those of the PDF subgrids, the
threshold knots duplicated.  Only inputs are produced here.
"""
import math
from dataclasses import dataclass

import numpy as np

from .configs import C1

ALPHA_MZ, MZ = 0.118, 91.1876
M_C, M_B = C1["q_edges"][1], C1["q_edges"][2]


@dataclass
class AlphasTable:
    q2_knots: list   # per subgrid, ascending; threshold knots duplicated
    values: list     # per subgrid, alpha_s at the knots


def _b0(nf):
    return (33.0 - 2.0 * nf) / (12.0 * math.pi)


def alphas_exact(q2):
    """The continuous one-loop function the table samples (input level)."""
    q2 = np.asarray(q2, dtype=np.float64)
    inv_b = 1.0 / ALPHA_MZ + _b0(5) * math.log(M_B**2 / MZ**2)
    inv_c = inv_b + _b0(4) * math.log(M_C**2 / M_B**2)
    inv = np.where(q2 >= M_B**2, 1.0 / ALPHA_MZ + _b0(5) * np.log(q2 / MZ**2),
                   np.where(q2 >= M_C**2, inv_b + _b0(4) * np.log(q2 / M_B**2),
                            inv_c + _b0(3) * np.log(q2 / M_C**2)))
    return 1.0 / inv


def synthetic_alphas(grid):
    return AlphasTable([np.array(q, dtype=np.float64) for q in grid.q2_knots],
                       [alphas_exact(np.array(q, dtype=np.float64)) for q in grid.q2_knots])

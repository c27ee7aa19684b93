"""Query points for PDF interpolation: x and Q log-uniform (seeded)."""
import numpy as np

from .configs import C1


def pdf_queries(n, seed=None, cfg=C1, q_min=None, q_max=None, x_min=None, x_max=None):
    """Return (x, q2) float64 arrays of length n, log-uniform in x and Q.

    Defaults: x in [1e-9, 1], Q in [1.65, 1e5] GeV, seed 0xC1.
    """
    rng = np.random.default_rng(cfg["query_seed"] if seed is None else seed)
    x_min = cfg["x_min"] if x_min is None else x_min
    x_max = cfg["x_max"] if x_max is None else x_max
    q_min = cfg["query_q_min"] if q_min is None else q_min
    q_max = cfg["query_q_max"] if q_max is None else q_max
    lx = rng.uniform(np.log(x_min), np.log(x_max), n)
    lq = rng.uniform(np.log(q_min), np.log(q_max), n)
    x = np.minimum(np.exp(lx), x_max)
    x = np.maximum(x, x_min)
    q2 = np.exp(2.0 * lq)
    q2 = np.clip(q2, q_min ** 2, q_max ** 2)
    return x, q2


def fk_points(cfg):
    """The C7 points: x log-spaced in [x_lo, x_hi], all at Q^2 = q^2."""
    x = np.exp(np.linspace(np.log(cfg["x_lo"]), np.log(cfg["x_hi"]), cfg["n_points"]))
    return x, np.full(cfg["n_points"], cfg["q"] ** 2)

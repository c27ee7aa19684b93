"""Specifications of the batched workload: many integrals, uneven shapes.

Families (integrand kinds) and their parameter vectors:

  GAUSS      params = [centre_0..centre_{d-1}, sigma_0..sigma_{d-1}]
  GENZ_OSC   params = [w_1, c_0..c_{d-1}]        (Genz oscillatory)
  GENZ_PEAK  params = [w_0..w_{d-1}, c_0..c_{d-1}] (Genz product peak)

Genz's difficulty parameters c are drawn U(0,1) and rescaled to a fixed
sum (4.5 oscillatory, 7.25 product peak), as is customary for that family.
"""
from dataclasses import dataclass

import numpy as np

from .configs import C3

GAUSS, GENZ_OSC, GENZ_PEAK, TTBAR = 0, 1, 2, 3
FAMILY_NAMES = {GAUSS: "gauss", GENZ_OSC: "genz_osc", GENZ_PEAK: "genz_peak", TTBAR: "ttbar"}


@dataclass
class BatchSpec:
    kind: int
    dim: int
    n: int
    params: np.ndarray
    stream: int


def gauss_params(dim, centre, sigma):
    c = np.broadcast_to(np.asarray(centre, dtype=np.float64), (dim,))
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (dim,))
    return np.concatenate([c, s])


def batch_specs(cfg=C3, n_integrals=None, n_scale=1.0, seed=None):
    """Return the list of BatchSpec of the batched workload (seeded).

    n_scale multiplies every sample count (for small test versions).
    """
    rng = np.random.default_rng(cfg["seed"] if seed is None else seed)
    m = cfg["n_integrals"] if n_integrals is None else n_integrals
    specs = []
    for i in range(m):
        d = int(rng.integers(cfg["dim_min"], cfg["dim_max"] + 1))
        n = int(round(np.exp(rng.uniform(np.log(cfg["n_min"]), np.log(cfg["n_max"])))))
        n = max(1, int(round(n * n_scale)))
        kind = int(rng.integers(0, 3))
        if kind == GAUSS:
            centre = rng.uniform(0.3, 0.7, d)
            sigma = rng.uniform(0.05, 0.3, d)
            params = np.concatenate([centre, sigma])
        elif kind == GENZ_OSC:
            w1 = rng.uniform()
            c = rng.uniform(0.0, 1.0, d)
            c *= 4.5 / c.sum()
            params = np.concatenate([[w1], c])
        else:
            w = rng.uniform(0.0, 1.0, d)
            c = rng.uniform(0.0, 1.0, d)
            c *= 7.25 / c.sum()
            params = np.concatenate([w, c])
        specs.append(BatchSpec(kind=kind, dim=d, n=n, params=params.astype(np.float64), stream=i))
    return specs

"""Write the oracle regression fixtures of this folder.

The thesis prints no worked numeric example for the VEGAS path (its MC
chapter gives the estimators, its PDF chapter the interpolation rule and its
examples only timings), so the oracle is pinned by closed forms, brute force
and quadrature in tests/test_oracle_*.py.  These fixtures only freeze the
oracle's own values at a few inputs, so that a later change of its
arithmetic shows up as a failing test and has to be justified.  This script
calls only oracle/ and synth/.

Usage: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import drellyan, integrands, singletop, ttbar, vegas  # noqa: E402
from oracle.philox import sample_words  # noqa: E402
from synth import C0, C2, C5, C6, synthetic_pdf_grid  # noqa: E402

U = [[0.1, 0.2, 0.3], [0.5, 0.5, 0.5], [0.9, 0.05, 0.75], [0.33, 0.66, 0.99], [0.01, 0.99, 0.01]]


def build():
    grid = synthetic_pdf_grid()
    u = np.array(U)
    out = {
        "philox_words": {
            "note": "sample_words(seed, stream, iteration, [index], dim=4): the 4 words of one sample",
            "cases": [],
        },
        "ttbar_integrand_pb": ttbar.integrand(u, grid, C2["sqrt_s"], C2["m_top"], C2["alpha_s"],
                                              C2["gev2_to_pb"]).tolist(),
        "drellyan_integrand_pb": drellyan.integrand_from_config(u, grid, C5).tolist(),
        "singletop_integrand_pb": singletop.integrand_from_config(u, grid, C6).tolist(),
        "points": U,
    }
    for seed, it, stream, idx in [(0, 0, 0, 0), (2, 3, 7, 123456789), (2**63 + 5, 9, (1 << 22) + 1, 2**40 + 3)]:
        w = sample_words(seed, stream, it, np.array([idx], dtype=np.uint64), 4)
        out["philox_words"]["cases"].append({"seed": str(seed), "iteration": it, "stream": stream, "index": str(idx),
                                             "words": [int(x) for x in np.asarray(w).ravel()]})
    f = lambda x: integrands.gauss(x, np.full(4, C0["centre"]), np.full(4, C0["sigma"]))
    r = vegas.run(f, 4, C0["n_bins"], C0["alpha"], 3, 20000, seed=C0["seed"])
    out["vegas_gauss4_3x20000"] = {"mean": r["mean"], "sigma": r["sigma"], "chi2_dof": r["chi2_dof"]}
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_values.json"), "w") as fh:
        json.dump(build(), fh, indent=1)
        fh.write("\n")

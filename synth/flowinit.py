"""Initial weights of the coupling-flow networks (seeded inputs).

The caller supplies the list of parameter segments of its network as
(kind, fan_in, size) triples: kind "w" segments are He-normal with
standard deviation sqrt(2 / fan_in), kind "b" segments are zero, and kind
"z" segments (the output layer of each coupling network) are zero so that
the untrained flow is the identity map with unit density.
"""
import numpy as np


def he_init_segments(segments, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for kind, fan_in, size in segments:
        if kind == "w":
            parts.append(rng.standard_normal(size) * np.sqrt(2.0 / fan_in))
        elif kind in ("b", "z"):
            parts.append(np.zeros(size))
        else:
            raise ValueError(f"unknown segment kind {kind!r}")
    return np.concatenate(parts).astype(np.float32)

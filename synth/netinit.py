"""Seeded initial weights of the warm-start network (an input generator: it
draws random numbers and holds none of the network's arithmetic).

Layer shapes (name, input channels, output channels, level) in the order of
the flat parameter vector: per convolution W[27][cout][cin] then b[cout];
then the 1x1 head Wh[18][16] and bh[18].
"""
from __future__ import annotations

import numpy as np

NET_LAYERS = (
    ("e0a", 3, 16, 0), ("e0b", 16, 16, 0),
    ("e1a", 16, 32, 1), ("e1b", 32, 32, 1),
    ("e2a", 32, 64, 2), ("e2b", 64, 64, 2),
    ("b3a", 64, 64, 3), ("b3b", 64, 64, 3),
    ("d2a", 128, 64, 2), ("d2b", 64, 64, 2),
    ("d1a", 96, 32, 1), ("d1b", 32, 32, 1),
    ("d0a", 48, 16, 0), ("d0b", 16, 16, 0),
)
NET_OUT, NET_HEAD_IN = 18, 16


def init_params(seed: int) -> np.ndarray:
    """He-normal convolution weights (std sqrt(2 / (27 cin))), biases N(0,
    0.01), head weights N(0, 0.1 / 4), head bias zero; FP64."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, _ in NET_LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), 27 * co * ci))
        parts.append(rng.normal(0.0, 0.01, co))
    parts.append(rng.normal(0.0, 0.1 / np.sqrt(NET_HEAD_IN), NET_OUT * NET_HEAD_IN))
    parts.append(np.zeros(NET_OUT))
    return np.concatenate(parts)

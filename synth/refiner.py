"""Seeded initial parameters of the pose refiner MLP (inputs of the tests and
the benchmark): Kaiming-normal weights (std sqrt(2 / fan_in)), zero biases,
an all-zero last layer, float32, in the flat per-scene layout W1, b1, ...,
W6, b6 with W_k stored out x in, row-major.  Random numbers only."""
from __future__ import annotations

import numpy as np

SHAPES = [(128, 12), (128, 128), (128, 128), (128, 128), (128, 128), (12, 128)]
N_PARAMS = sum(o * i + o for o, i in SHAPES)


def offsets():
    out, o = [], 0
    for rows, cols in SHAPES:
        out.append((o, o + rows * cols))
        o += rows * cols + rows
    return out


def init_params(rng: np.random.Generator, n_scenes: int = 1, last_std: float = 0.0,
                bias_std: float = 0.0) -> np.ndarray:
    """(n_scenes, N_PARAMS) float32.  last_std / bias_std > 0 give a non-zero
    last layer / biases (test states away from the initial one)."""
    th = np.zeros((n_scenes, N_PARAMS), np.float32)
    for s in range(n_scenes):
        for k, ((wo, bo), (rows, cols)) in enumerate(zip(offsets(), SHAPES)):
            std = np.sqrt(2.0 / cols) if k < len(SHAPES) - 1 else last_std
            if std > 0:
                th[s, wo:bo] = rng.normal(0.0, std, rows * cols)
            if bias_std > 0:
                th[s, bo:bo + rows] = rng.normal(0.0, bias_std, rows)
    return th

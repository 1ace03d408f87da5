"""Seeded initial weights of the step-scale network (random inputs shared by the
library and the oracle; no method arithmetic).

Layout (741 values): W1 [32][17] row-major, b1 [32], W2 [5][32] row-major, b2 [5].
He-normal first layer, small second layer, zero biases.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 17, 32, 5


def init_params(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_HID, N_IN)) * np.sqrt(2.0 / N_IN)
    W2 = rng.standard_normal((N_OUT, N_HID)) * 0.01
    return np.concatenate([W1.ravel(), np.zeros(N_HID), W2.ravel(), np.zeros(N_OUT)]).astype(np.float32)


def random_features(n: int, seed: int = 1) -> np.ndarray:
    """Feature rows in the range the features take ([-3, 3], signs +-1)."""
    rng = np.random.default_rng(seed)
    F = rng.uniform(-1.5, 0.5, (n, N_IN))
    for c in (2, 4, 7):
        F[:, c] = np.where(rng.random(n) < 0.8, 1.0, -1.0)
    return F.astype(np.float32)

"""Seeded initial parameters of the learned surrogate (random numbers only)."""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

N_FEAT, H1, H2 = 256, 128, 128


def surrogate_weights(seed: int = 0, scale: float = 1.0) -> Dict[str, np.ndarray]:
    """Glorot-normal weight matrices, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.normal(0, scale * math.sqrt(2.0 / (N_FEAT + H1)), (N_FEAT, H1)),
        "b1": np.zeros(H1),
        "W2": rng.normal(0, scale * math.sqrt(2.0 / (H1 + H2)), (H1, H2)),
        "b2": np.zeros(H2),
        "w3": rng.normal(0, scale * math.sqrt(2.0 / (H2 + 1)), (H2,)),
        "b3": np.zeros(1),
    }

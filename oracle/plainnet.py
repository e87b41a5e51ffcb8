"""FP64 plaintext network: the accuracy reference (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Dense layers with bias and the square activation between them (paper,
"Non-convolutional layers": bias and polynomial activation collapsed into a
per-feature polynomial; the activation here is x^2).
"""
from __future__ import annotations

import numpy as np


def forward(x: np.ndarray, weights: list[np.ndarray], biases: list[np.ndarray]) -> np.ndarray:
    h = np.asarray(x, dtype=np.float64)
    for li, (W, b) in enumerate(zip(weights, biases)):
        h = W.astype(np.float64) @ h + b.astype(np.float64)
        if li + 1 < len(weights):
            h = h * h
    return h


def predict(y: np.ndarray) -> int:
    """Arg-max with ties to the lowest index."""
    return int(np.argmax(y))

"""FP64 plaintext network: the accuracy reference (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Dense layers with bias and a per-feature polynomial activation between them
(paper, "Non-convolutional layers": bias, batch normalisation and the
trained quadratic activation collapse into one polynomial per feature, applied
slot-wise; Methods, "Network architecture": ReLU replaced by a quadratic whose
coefficients are trained).  Default activation: x^2; with acts, feature k of
activation i is a_k x^2 + b_k x + c_k.
"""
from __future__ import annotations

import numpy as np


def forward(x: np.ndarray, weights: list[np.ndarray], biases: list[np.ndarray], acts=None) -> np.ndarray:
    """acts: None (x^2 after every layer but the last) or, per activation, a
    tuple (a, b, c) of per-feature coefficient vectors."""
    h = np.asarray(x, dtype=np.float64)
    for li, (W, b) in enumerate(zip(weights, biases)):
        h = W.astype(np.float64) @ h + b.astype(np.float64)
        if li + 1 < len(weights):
            if acts is None:
                h = h * h
            else:
                a2, a1, a0 = (np.asarray(v, dtype=np.float64) for v in acts[li])
                h = a2 * h * h + a1 * h + a0
    return h


def predict(y: np.ndarray) -> int:
    """Arg-max with ties to the lowest index."""
    return int(np.argmax(y))

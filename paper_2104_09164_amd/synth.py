"""Seeded synthetic inputs of the encrypted-inference workloads.

Holds no arithmetic of the method: only random draws with numpy's PCG64
(seeded per object), shared by tests, the benchmark and the oracle-side test
drivers.  The paper's inputs are skeleton tensors of 2 x 32 x 15 min-max
normalised joint coordinates, padded and replicated into the slots (Methods,
"Data encryption", "Data preprocessing"); the stand-ins here are uniform in
[-1, 1] with the same padded widths, and weights are N(0, sigma^2).
"""
from __future__ import annotations

import numpy as np

SEED_KEYS, SEED_WEIGHTS, SEED_STEPS = 1, 2, 3


def request_input(width: int, request: int) -> np.ndarray:
    """Input vector of request r: U[-1, 1]^width, seed 1000 + r."""
    return np.random.default_rng(1000 + request).uniform(-1.0, 1.0, width)


def request_seed(request: int) -> int:
    """Encryption seed of request r."""
    return 5000 + request


def network_weights(layers, sigma: float, seed: int = SEED_WEIGHTS):
    """Weights W_i (m x n) and biases b_i (m) ~ N(0, sigma^2) for layers [(m, n, n1), ...]."""
    rng = np.random.default_rng(seed)
    Ws = [rng.normal(0.0, sigma, (m, n)) for m, n, _ in layers]
    bs = [rng.normal(0.0, sigma, m) for m, _, _ in layers]
    return Ws, bs


def activation_coeffs(layers, seed: int = SEED_WEIGHTS + 10):
    """Per-feature quadratic activations (a, b, c) after every layer but the
    last, shaped like a trained quadratic stand-in for ReLU on [-1, 1]:
    a ~ U[0.2, 0.6], b ~ U[0.3, 0.7], c ~ U[0, 0.2] (a bounded away from 0)."""
    rng = np.random.default_rng(seed)
    return [(rng.uniform(0.2, 0.6, m), rng.uniform(0.3, 0.7, m), rng.uniform(0.0, 0.2, m))
            for m, _, _ in layers[:-1]]


def uniform_residues(primes, n: int, shape_prefix=(), seed: int = 0) -> np.ndarray:
    """uint64 array shape_prefix + [len(primes)][n], each row uniform in [0, q)."""
    rng = np.random.default_rng(seed)
    out = np.empty(tuple(shape_prefix) + (len(primes), n), dtype=np.uint64)
    for i, q in enumerate(primes):
        out[..., i, :] = rng.integers(0, q, tuple(shape_prefix) + (n,), dtype=np.uint64)
    return out


def rotation_steps_random(count: int, slots: int, seed: int = SEED_STEPS) -> list[int]:
    """`count` distinct steps drawn uniformly from [1, slots)."""
    rng = np.random.default_rng(seed)
    return sorted(int(v) for v in rng.choice(np.arange(1, slots), size=count, replace=False))


def encryption_noise(n: int, seed: int) -> np.ndarray:
    """Random polynomials of one public-key encryption, int32 [3][n]:
    v with coefficients uniform in {-1, 0, 1}, then e0 and e1, rounded
    N(0, 3.2^2) clipped to |e| <= 19."""
    rng = np.random.default_rng(seed)
    v = rng.integers(-1, 2, n)
    e = np.clip(np.rint(rng.normal(0.0, 3.2, (2, n))), -19, 19)
    return np.concatenate([v[None, :], e]).astype(np.int32)


def slot_vectors(count: int, slots: int, seed: int) -> np.ndarray:
    """`count` complex slot vectors, real and imaginary parts U[-1, 1]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (count, slots)) + 1j * rng.uniform(-1.0, 1.0, (count, slots))

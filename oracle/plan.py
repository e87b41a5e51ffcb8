"""Dense-layer plan: diagonals, baby-step pre-rotation, rotation steps (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A dense layer y = W x + b (W is m x n, m | n, n | N/2, powers of two) acts on
a ciphertext whose slots hold x replicated with period n (paper, "Data
encryption": zero-pad to a power of two and replicate copies across all N/2
slots so rotations wrap correctly).  With hybrid diagonals
    d_k[s] = W[s mod m][(s + k) mod n],  s < n, k < m,
sum_k d_k * rho^k(x) summed over the n/m shifts s, s+m, ... gives Wx with
period m; the shifts are summed by rotate-and-sum (paper, "Fast homomorphic
convolutions", recursive rotate-and-sum in log steps).

Baby-step/giant-step split (paper, "Algorithmic and cryptographic
optimizations", baby-step rewriting with rho^(a+b) = rho^a o rho^b):
k = n1*j + i, i < n1, j < n2 = m/n1, and the plaintext for (j, i) is
rho^(-n1*j)(d_k): slot s holds d_k[(s - n1*j) mod n].
"""
from __future__ import annotations

import numpy as np


def check_shape(m: int, n: int, n1: int, slots: int) -> None:
    def pow2(v):
        return v > 0 and v & (v - 1) == 0
    if not (pow2(m) and pow2(n) and pow2(n1)):
        raise ValueError("m, n, n1 must be powers of two")
    if n % m or m % n1 or slots % n:
        raise ValueError("need m | n, n1 | m and n | N/2")


def diagonals(W: np.ndarray) -> np.ndarray:
    """d[k][s] = W[s mod m][(s + k) mod n] for k < m, s < n."""
    m, n = W.shape
    s = np.arange(n)
    return np.stack([W[s % m, (s + k) % n] for k in range(m)])


def plaintext_slots(W: np.ndarray, n1: int, slots: int) -> np.ndarray:
    """Slot vectors [m][slots] of the pre-rotated diagonals, period n."""
    m, n = W.shape
    check_shape(m, n, n1, slots)
    d = diagonals(W)
    out = np.empty((m, slots))
    s = np.arange(slots)
    for k in range(m):
        j = k // n1
        out[k] = d[k][(s - n1 * j) % n]
    return out


def bias_slots(b: np.ndarray, slots: int) -> np.ndarray:
    """Bias replicated with period m."""
    m = len(b)
    return np.asarray(b, dtype=np.float64)[np.arange(slots) % m]


def input_slots(x: np.ndarray, slots: int) -> np.ndarray:
    """Input replicated with period n."""
    n = len(x)
    return np.asarray(x, dtype=np.float64)[np.arange(slots) % n]


def rotate_sum_steps(m: int, n: int, rs_bits: int = 0) -> list[int]:
    """Rotation amounts of the rotate-and-sum that leaves period m from period
    n.  rs_bits = 0: sequential n/2, n/4, .., m.  rs_bits = b > 0: hoisted
    groups over the log2(n/m) bits of the shift index, b bits at a time from
    the most significant; a group of b' bits with base shift t uses k t for
    0 < k < 2^b'.  (b = 1 gives the sequential amounts.)"""
    if rs_bits <= 0:
        steps, t = [], n // 2
        while t >= m:
            steps.append(t)
            t //= 2
        return steps
    left = (n // m).bit_length() - 1
    steps = []
    while left > 0:
        b = min(rs_bits, left)
        left -= b
        t = m << left
        steps += [k * t for k in range(1, 1 << b)]
    return steps


def rotation_steps(m: int, n: int, n1: int, rs_bits: int = 0) -> list[int]:
    """Baby steps 1..n1-1, giant steps n1*j (j < m/n1), rotate-and-sum steps."""
    steps = list(range(1, n1)) + [n1 * j for j in range(1, m // n1)]
    return steps + rotate_sum_steps(m, n, rs_bits)


def op_counts(m: int, n: int, n1: int) -> dict:
    """Key switches, MultPlain and hoisted ModUp groups of one dense layer."""
    n2 = m // n1
    rs = 0
    t = n // 2
    while t >= m:
        rs += 1
        t //= 2
    return {"rotations": (n1 - 1) + (n2 - 1) + rs, "multplain": m, "hoisted_modup": 1 if n1 > 1 else 0,
            "baby": n1 - 1, "giant": n2 - 1, "rotate_and_sum": rs}

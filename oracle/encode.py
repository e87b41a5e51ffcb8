"""CKKS encoder and decoder in FP64 (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Slot j of a plaintext polynomial m(X) in R[X]/(X^N+1) is its value at
zeta^(5^j mod 2N), zeta = exp(i*pi/N); slot j+N/2 would be the conjugate
(exponent -5^j).  With this ordering the automorphism X -> X^(5^r) rotates the
slot vector left by r, which is the paper's rho^r ("Single-channel
homomorphic convolutions": rho^l is a left rotation by l positions).

The paper does not state the encoding rounding; coefficients are scaled by
Delta and rounded half away from zero.
"""
from __future__ import annotations

import numpy as np


def slot_exponents(n: int) -> np.ndarray:
    """e_j = 5^j mod 2N for j < N/2."""
    e = np.empty(n // 2, dtype=np.int64)
    v = 1
    for j in range(n // 2):
        e[j] = v
        v = v * 5 % (2 * n)
    return e


def round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def embed_inverse(z: np.ndarray, n: int) -> np.ndarray:
    """Real coefficients m_k = (2/N) Re sum_j z_j zeta^(-5^j k), via one FFT.

    v over odd exponents t = 2u+1: v[u] = z_j if t = 5^j, conj(z_j) if t = -5^j
    (mod 2N); then m_k = Re(zeta^-k * fft(v)[k]) / N.
    """
    z = np.asarray(z, dtype=np.complex128)
    assert z.shape == (n // 2,)
    e = slot_exponents(n)
    v = np.zeros(n, dtype=np.complex128)
    v[(e - 1) // 2] = z
    v[(2 * n - e - 1) // 2] = np.conj(z)
    k = np.arange(n)
    zeta_mk = np.exp(-1j * np.pi * k / n)
    return np.real(zeta_mk * np.fft.fft(v)) / n


def embed_inverse_direct(z: np.ndarray, n: int) -> np.ndarray:
    """O(N^2) direct sum of the same formula (cross-check of the FFT form)."""
    z = np.asarray(z, dtype=np.complex128)
    e = slot_exponents(n)
    k = np.arange(n)
    ang = -np.pi * np.outer(e, k) / n            # [slot][k]
    return (2.0 / n) * np.real((z[:, None] * np.exp(1j * ang)).sum(axis=0))


def encode_coeffs(z, scale: float, n: int, direct: bool = False) -> np.ndarray:
    """Integer coefficients M_k = round(scale * m_k), as exact integers held in
    FP64 (the product scale * m_k is formed in FP64, then rounded half away
    from zero).  Below 2^53 every integer is exact; above it (a bias encoded
    at scale Delta^2) the FP64 value is itself the integer used."""
    m = embed_inverse_direct(z, n) if direct else embed_inverse(z, n)
    M = round_half_away(m * scale)
    if not np.all(np.isfinite(M)):
        raise OverflowError("encoded coefficient is not finite")
    return M


def to_rns(coeffs: np.ndarray, primes) -> np.ndarray:
    """Residues [len(primes)][N] (uint64) of integer coefficients (int64 or
    integral FP64); exact for any magnitude."""
    c = np.asarray(coeffs)
    if c.dtype.kind == "f" and np.all(np.abs(c) < 2.0 ** 62) or c.dtype.kind in "iu":
        c = c.astype(np.int64)
        return np.stack([np.mod(c, np.int64(q)).astype(np.uint64) for q in primes])
    ints = [int(v) for v in c]                       # exact: every finite double is an integer here
    return np.stack([np.array([v % q for v in ints], dtype=np.uint64) for q in primes])


def encode(z, scale: float, primes, n: int) -> np.ndarray:
    """Plaintext residues over ``primes`` (level-aware: pass q_0..q_l only)."""
    return to_rns(encode_coeffs(z, scale, n), primes)


def crt_lift(res: np.ndarray, primes) -> list[int]:
    """Centred integer in (-Q/2, Q/2] of every coefficient from its residues."""
    Q = 1
    for q in primes:
        Q *= q
    acc = np.zeros(res.shape[1], dtype=object)
    for i, q in enumerate(primes):
        qi_hat = Q // q
        c = qi_hat * pow(qi_hat % q, -1, q)
        acc = acc + res[i].astype(object) * c
    acc = acc % Q
    half = Q // 2
    return [int(v) - Q if int(v) > half else int(v) for v in acc]


def embed(m: np.ndarray, n: int) -> np.ndarray:
    """Slots z_j = m(zeta^(5^j)) of real coefficients m (length N)."""
    m = np.asarray(m, dtype=np.float64)
    k = np.arange(n)
    w = m * np.exp(1j * np.pi * k / n)          # m_k zeta^k
    vals = np.fft.ifft(w) * n                   # vals[u] = sum_k m_k zeta^(k (2u+1))
    e = slot_exponents(n)
    return vals[(e - 1) // 2]


def decode(res: np.ndarray, scale: float, primes, n: int) -> np.ndarray:
    """Complex slots of a plaintext given by residues over ``primes``."""
    ints = crt_lift(res, primes)
    m = np.array([float(v) for v in ints]) / scale
    return embed(m, n)

"""Multi-channel homomorphic convolution (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper, Methods: "Single-channel homomorphic convolutions" (a convolution as
rotations of the input, products with plaintexts holding the filter weights,
and a sum) and the multi-channel form that follows it: c channels of length
L are packed into one ciphertext at slot distance `dist` (channel l of the
ciphertext in slots l dist .. l dist + L - 1, the rest of its block zero, the
block of c channels replicated across the slots); output block j of c output
channels is
    sum_i sum_l sum_k MultPlain(rho^{r_k + dist l}(ct_i), pt_{i,j,k,l}),
evaluated in the paper's baby-step strategy ("Algorithmic and cryptographic
optimizations", (iii)):
    sum_l rho^{dist l}( sum_{i,k} MultPlain(rho^{r_k}(ct_i), rho^{-dist l}(pt_{i,j,k,l})) ).
Here the convolution is 1-D with odd kernel width f, r_k = k - floor(f/2),
zero padding (dist >= L + floor(f/2)), and c input and c output channels per
ciphertext.  pt_{i,j,k,l} holds in block b, positions t < L, the weight
W[j c + b][i c + (b + l) mod c][k]; zero at t >= L (so the outputs' padding
stays zero).
"""
from __future__ import annotations

import numpy as np


def conv1d_fp64(X: np.ndarray, W: np.ndarray) -> np.ndarray:
    """out[o][t] = sum_{ch, k} W[o][ch][k] X[ch][t + k - f//2], zero outside [0, L)."""
    c_in, L = X.shape
    c_out, c_in2, f = W.shape
    assert c_in2 == c_in
    h = f // 2
    Xp = np.zeros((c_in, L + 2 * h))
    Xp[:, h:h + L] = X
    out = np.zeros((c_out, L))
    for k in range(f):
        out += W[:, :, k] @ Xp[:, k:k + L]
    return out


def pack(X: np.ndarray, c: int, dist: int, slots: int) -> list[np.ndarray]:
    """Slot vectors of the input ciphertexts: channels i c .. i c + c - 1 in ciphertext i."""
    c_in, L = X.shape
    assert c_in % c == 0 and L <= dist and slots % (c * dist) == 0
    out = []
    for i in range(c_in // c):
        block = np.zeros(c * dist)
        for l in range(c):
            block[l * dist:l * dist + L] = X[i * c + l]
        out.append(np.tile(block, slots // (c * dist)))
    return out


def unpack(v: np.ndarray, c: int, dist: int, L: int) -> np.ndarray:
    """Channels of one output ciphertext (its first block)."""
    return np.stack([v[l * dist:l * dist + L] for l in range(c)])


def rotations(f: int, c: int, dist: int) -> tuple[list[int], list[int]]:
    """Baby amounts r_k = k - floor(f/2) and giant amounts dist l, l < c."""
    return [k - f // 2 for k in range(f)], [dist * l for l in range(c)]


def plaintext_slots(W: np.ndarray, c: int, dist: int, L: int, slots: int) -> np.ndarray:
    """Slot vectors pt[g][j][i][k] = rho^{-dist g}(pt_{i,j,k,g}) as float64
    [c][n_out][n_in][f][slots] (giant index g = channel offset l)."""
    c_out, c_in, f = W.shape
    n_in, n_out = c_in // c, c_out // c
    out = np.zeros((c, n_out, n_in, f, slots))
    for g in range(c):
        for j in range(n_out):
            for i in range(n_in):
                for k in range(f):
                    block = np.zeros(c * dist)
                    for b in range(c):
                        block[b * dist:b * dist + L] = W[j * c + b, i * c + (b + g) % c, k]
                    v = np.tile(block, slots // (c * dist))
                    out[g, j, i, k] = np.roll(v, dist * g)      # rho^{-dist g}: v[s - dist g]
    return out


def encode_plaintexts(oracle, slot_vecs: np.ndarray, scale: float, level: int) -> np.ndarray:
    """uint64 [n_giant][n_out][n_in][n_baby][level+1][N]: each slot vector encoded at `scale`."""
    shp = slot_vecs.shape[:4]
    flat = [oracle.encode(v, scale, level) for v in slot_vecs.reshape(-1, slot_vecs.shape[-1])]
    return np.stack(flat).reshape(shp + flat[0].shape)


def slot_model(xs: list[np.ndarray], pt_slots: np.ndarray, baby: list[int], giant: list[int]) -> list[np.ndarray]:
    """The baby-step formula on plain slot vectors (rho^r = left rotation by r)."""
    n_giant, n_out, n_in, n_baby = pt_slots.shape[:4]
    outs = []
    for j in range(n_out):
        z = np.zeros_like(xs[0])
        for g in range(n_giant):
            s = sum(pt_slots[g, j, i, b] * np.roll(xs[i], -baby[b]) for i in range(n_in) for b in range(n_baby))
            z = z + np.roll(s, -giant[g])
        outs.append(z)
    return outs

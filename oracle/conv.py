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


# ----------------------------------------------------------------------------
# Fast convolution (paper, "Fast homomorphic convolutions", merge-and-conquer).
# Inputs are punctured: channel l of ciphertext i holds its map of length Lp
# at positions nP u (u < Lp) of block l, arbitrary junk elsewhere (as left by
# a pooling step).  (i) Pre: each group of nP ciphertexts i = a nP + p is
# masked to its valid positions and shifted right by p, and the group summed:
# merged a holds input ciphertext a nP + p at positions nP u + p.  (ii) The
# multi-channel convolution on the n_in / nP merged ciphertexts, kernel
# offsets nP r_k, each position nP u + p weighted for input ciphertext
# a nP + p.  (iii) Post: rotate-and-sum by nP/2, .., 1 collects the nP partial
# sums of position nP u onto it; the outputs are punctured the same way.

def pack_punctured(X: np.ndarray, c: int, dist: int, nP: int, slots: int, rng) -> list[np.ndarray]:
    """Punctured input ciphertexts (junk U[-1, 1] at the invalid positions)."""
    c_in, Lp = X.shape
    assert nP * Lp <= dist and c_in % c == 0
    out = []
    for i in range(c_in // c):
        block = rng.uniform(-1, 1, c * dist)
        for l in range(c):
            block[l * dist + nP * np.arange(Lp)] = X[i * c + l]
        out.append(np.tile(block, slots // (c * dist)))
    return out


def merge_plaintext_slots(c: int, dist: int, Lp: int, nP: int, slots: int) -> tuple[np.ndarray, list[int]]:
    """Pre step as a linear transform of nP inputs into one output:
    out = sum_p rho^{-p}(mask (.) ct_p): slot vectors pt[g][0][i][0] (= mask
    when i == g, zero otherwise; the mask moves with its ciphertext) and giant
    amounts -p."""
    block = np.zeros(c * dist)
    for l in range(c):
        block[l * dist + nP * np.arange(Lp)] = 1.0
    mask = np.tile(block, slots // (c * dist))
    pts = np.zeros((nP, 1, nP, 1, slots))
    for g in range(nP):
        pts[g, 0, g, 0] = mask
    return pts, [-g for g in range(nP)]


def fast_plaintext_slots(W: np.ndarray, c: int, dist: int, Lp: int, nP: int, slots: int) -> np.ndarray:
    """Conv step on the merged ciphertexts: slot vectors pt[g][j][a][k], block
    b position nP u + p carrying W[j c + b][(a nP + p) c + (b + g) mod c][k],
    pre-rotated by -dist g."""
    c_out, c_in, f = W.shape
    n_in, n_out = c_in // c, c_out // c
    assert n_in % nP == 0 and nP * (Lp + f // 2) <= dist       # zero gap for the kernel offsets
    out = np.zeros((c, n_out, n_in // nP, f, slots))
    u = np.arange(Lp)
    for g in range(c):
        for j in range(n_out):
            for a in range(n_in // nP):
                for k in range(f):
                    block = np.zeros(c * dist)
                    for b in range(c):
                        for p in range(nP):
                            block[b * dist + nP * u + p] = W[j * c + b, (a * nP + p) * c + (b + g) % c, k]
                    out[g, j, a, k] = np.roll(np.tile(block, slots // (c * dist)), dist * g)
    return out


def unpack_punctured(v: np.ndarray, c: int, dist: int, Lp: int, nP: int) -> np.ndarray:
    return np.stack([v[l * dist + nP * np.arange(Lp)] for l in range(c)])


def fast_rotations(f: int, c: int, dist: int, nP: int) -> dict:
    """Rotation amounts of the three steps: pre giants -p, conv babies nP r_k
    and giants dist l, post nP/2, .., 1."""
    post, t = [], nP // 2
    while t >= 1:
        post.append(t)
        t //= 2
    return {"pre": [-p for p in range(nP)], "baby": [nP * (k - f // 2) for k in range(f)],
            "giant": [dist * l for l in range(c)], "post": post}


def fast_conv(o, cts: list, pre_pts: np.ndarray, conv_pts: np.ndarray, rot: dict, scale: float, keys, only=None):
    """The three steps on the oracle: merged_a = Rescale(pre(cts of group a)),
    z_j = conv(merged) (pre-rotated conv plaintexts at the next level),
    z_j <- z_j + rho^t(z_j) for the post amounts, then Rescale."""
    nP = len(rot["pre"])
    merged = [o.rescale(o.linear(cts[a * nP:(a + 1) * nP], pre_pts, [0], rot["pre"], scale, keys)[0])
              for a in range(len(cts) // nP)]
    outs = o.linear(merged, conv_pts, rot["baby"], rot["giant"], scale, keys, only=only)
    res = []
    for z in outs:
        for t in rot["post"]:
            z = o.add(z, o.rotate(z, t, keys))
        res.append(o.rescale(z))
    return merged, res

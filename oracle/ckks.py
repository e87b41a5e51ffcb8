"""ctypes driver of the C++ oracle core (``cpp/ckks_oracle.cpp``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Client side (paper, Results/Methods: the monitoring provider generates the
keys and sends only evaluation keys to the cloud; users encrypt with the
public key; the provider decrypts the single output ciphertext): keygen,
encrypt, decrypt.  Server side, evaluated exactly as the GPU library must:
add, MultPlain, rescale, rotate (hoisted key switching), square
(relinearised), dense (baby-step/giant-step + rotate-and-sum + bias) and the
whole network with lazy rescaling (one rescale per layer and per square).

Scales are IEEE doubles updated only by *Delta_w, by squaring and by /q_l, in
that order, so the GPU reproduces them bit for bit.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import encode as enc
from . import plan as planmod
from .params import Params

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpp", "ckks_oracle.cpp")
# ORACLE_SANITIZE=1: the same source built with AddressSanitizer and
# UndefinedBehaviorSanitizer (errors fatal), for a test run of the pins under
# them (the process must preload the ASan runtime).
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "cpp", "liboracle_san.so" if _SANITIZE else "liboracle.so")
_FLAGS = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
          if _SANITIZE else ["-O2"])

U64P = C.POINTER(C.c_uint64)
I64P = C.POINTER(C.c_int64)
I32P = C.POINTER(C.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle core with g++ (plain C++17, OpenMP over limbs)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", *_FLAGS, "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.orc_ctx_new.restype = C.c_void_p
        L.orc_ctx_new.argtypes = [C.c_int, U64P, C.c_int, U64P, C.c_int, C.c_int]
        L.orc_ctx_free.argtypes = [C.c_void_p]
        L.orc_psi.restype = C.c_uint64
        L.orc_psi.argtypes = [C.c_void_p, C.c_int]
        L.orc_sample_ternary.argtypes = [C.c_uint64, C.c_int, I64P]
        L.orc_sample_gaussian.argtypes = [C.c_uint64, C.c_int, I64P]
        L.orc_sample_uniform.argtypes = [C.c_void_p, C.c_uint64, C.c_int, I32P, U64P]
        L.orc_derive_seed.restype = C.c_uint64
        L.orc_derive_seed.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_splitmix_first.restype = C.c_uint64
        L.orc_splitmix_first.argtypes = [C.c_uint64]
        L.orc_polymul.argtypes = [C.c_void_p, C.c_int, I32P, U64P, U64P, U64P]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = [C.c_int]
        L.orc_ntt_roundtrip.argtypes = [C.c_void_p, C.c_int, I32P, U64P]
        L.orc_automorph.argtypes = [C.c_void_p, C.c_int, I32P, C.c_uint64, U64P, U64P]
        L.orc_keygen_public.argtypes = [C.c_void_p, I64P, C.c_uint64, U64P]
        L.orc_keygen_switch.argtypes = [C.c_void_p, I64P, U64P, C.c_uint64, U64P]
        L.orc_encrypt.argtypes = [C.c_void_p, U64P, U64P, C.c_uint64, U64P]
        L.orc_encrypt_noise.argtypes = [C.c_void_p, U64P, U64P, C.c_int, I64P, I64P, I64P, U64P]
        L.orc_decrypt.argtypes = [C.c_void_p, I64P, U64P, C.c_int, U64P]
        L.orc_add.argtypes = [C.c_void_p, U64P, U64P, C.c_int, U64P]
        L.orc_add_plain.argtypes = [C.c_void_p, U64P, U64P, C.c_int, U64P]
        L.orc_mult_plain.argtypes = [C.c_void_p, U64P, U64P, C.c_int, U64P]
        L.orc_rescale.argtypes = [C.c_void_p, U64P, C.c_int, U64P]
        L.orc_modup.argtypes = [C.c_void_p, U64P, C.c_int, C.c_int, U64P]
        L.orc_moddown.argtypes = [C.c_void_p, U64P, C.c_int, U64P]
        L.orc_keyswitch.argtypes = [C.c_void_p, U64P, C.c_int, U64P, U64P]
        L.orc_galois_elt.restype = C.c_uint64
        L.orc_galois_elt.argtypes = [C.c_void_p, C.c_int64]
        L.orc_rotate.argtypes = [C.c_void_p, U64P, C.c_int, C.c_int64, U64P, U64P]
        L.orc_square.argtypes = [C.c_void_p, U64P, C.c_int, U64P, U64P]
        L.orc_rotate_ext.argtypes = [C.c_void_p, U64P, C.c_int, C.c_int64, U64P, U64P]
        L.orc_dense_ex.restype = C.c_int
        L.orc_dense_ex.argtypes = [C.c_void_p, U64P, C.c_int, C.c_int, C.c_int, C.c_int, U64P, U64P,
                                   C.c_int, I64P, C.POINTER(U64P), C.c_int, C.c_int, U64P]
        for f in (L.orc_dense, L.orc_dense_qp):
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, U64P, C.c_int, C.c_int, C.c_int, C.c_int, U64P, U64P,
                          C.c_int, I64P, C.POINTER(U64P), U64P]
        _lib = L
    return _lib


def _p(a: np.ndarray, t=U64P):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(t)


# Seed tags of the sampled client objects.
TAG_SECRET = 0x5EC
TAG_PUBLIC = 0x9B
TAG_RELIN = 0x4E1


def tag_rotation(r: int) -> int:
    return (0x40 << 32) | (r & 0xFFFFFFFF)


@dataclass
class Ciphertext:
    data: np.ndarray          # uint64 [2][level+1][N], coefficient form
    level: int
    scale: float

    def copy(self):
        return Ciphertext(self.data.copy(), self.level, self.scale)


@dataclass
class Keys:
    sk: np.ndarray            # int64 [N] ternary
    pk: np.ndarray            # uint64 [2][L+1][N]
    rlk: np.ndarray | None    # uint64 [dnum][2][L+1+K][N]
    rot: dict                 # step -> uint64 [dnum][2][L+1+K][N]


class Oracle:
    def __init__(self, params: Params):
        self.pr = params
        self.N = params.n
        L = lib()
        q = np.array(params.q, dtype=np.uint64)
        p = np.array(params.p, dtype=np.uint64)
        self._h = L.orc_ctx_new(params.log_n, _p(q), len(q), _p(p), len(p), params.alpha)
        self.L = L
        self.primes = list(params.q) + list(params.p)

    def __del__(self):
        try:
            self.L.orc_ctx_free(self._h)
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def qs(self, level: int) -> list[int]:
        return self.pr.q[: level + 1]

    def psi(self, i: int) -> int:
        return int(self.L.orc_psi(self._h, i))

    def galois(self, r: int) -> int:
        return int(self.L.orc_galois_elt(self._h, r))

    def _idx(self, n):
        return np.arange(n, dtype=np.int32)

    # ------------------------------------------------------------ sampling
    def secret(self, seed: int) -> np.ndarray:
        s = np.empty(self.N, dtype=np.int64)
        self.L.orc_sample_ternary(self.L.orc_derive_seed(seed, TAG_SECRET), self.N, _p(s, I64P))
        return s

    def _s_rns(self, s: np.ndarray) -> np.ndarray:
        return np.stack([np.mod(s, np.int64(q)).astype(np.uint64) for q in self.primes])

    def keygen(self, seed: int, steps=(), relin: bool = True) -> Keys:
        pr = self.pr
        s = self.secret(seed)
        pk = np.empty((2, pr.L + 1, self.N), dtype=np.uint64)
        self.L.orc_keygen_public(self._h, _p(s, I64P), self.L.orc_derive_seed(seed, TAG_PUBLIC), _p(pk))
        s_rns = self._s_rns(s)
        nt = len(self.primes)
        rlk = None
        if relin:
            s2 = np.empty_like(s_rns)
            self.L.orc_polymul(self._h, nt, _p(self._idx(nt), I32P), _p(s_rns), _p(s_rns), _p(s2))
            rlk = self.switch_key(s, s2, self.L.orc_derive_seed(seed, TAG_RELIN))
        rot = {}
        for r in steps:
            g = self.galois(r)
            sg = np.empty_like(s_rns)
            self.L.orc_automorph(self._h, nt, _p(self._idx(nt), I32P), g, _p(s_rns), _p(sg))
            rot[int(r)] = self.switch_key(s, sg, self.L.orc_derive_seed(seed, tag_rotation(int(r))))
        return Keys(s, pk, rlk, rot)

    def switch_key(self, s: np.ndarray, s_prime_rns: np.ndarray, seed: int) -> np.ndarray:
        pr = self.pr
        ksk = np.empty((pr.dnum, 2, len(self.primes), self.N), dtype=np.uint64)
        self.L.orc_keygen_switch(self._h, _p(s, I64P), _p(np.ascontiguousarray(s_prime_rns)), seed, _p(ksk))
        return ksk

    # ---------------------------------------------------- encode/encrypt
    def encode(self, z, scale: float, level: int) -> np.ndarray:
        return enc.encode(z, scale, self.qs(level), self.N)

    def encrypt(self, z, pk: np.ndarray, seed: int, scale: float | None = None) -> Ciphertext:
        pr = self.pr
        scale = pr.scale if scale is None else scale
        m = self.encode(z, scale, pr.L)
        ct = np.empty((2, pr.L + 1, self.N), dtype=np.uint64)
        self.L.orc_encrypt(self._h, _p(pk), _p(m), seed, _p(ct))
        return Ciphertext(ct, pr.L, scale)

    def encrypt_noise(self, m: np.ndarray, pk: np.ndarray, level: int, v, e0, e1, scale: float) -> Ciphertext:
        """Encryption of plaintext residues m ([level+1][N]) with the given
        random polynomials (v ternary, e0, e1 small): (v b + e0 + m, v a + e1)."""
        m = np.ascontiguousarray(m, dtype=np.uint64)
        assert m.shape == (level + 1, self.N)
        vs = [np.ascontiguousarray(x, dtype=np.int64) for x in (v, e0, e1)]
        assert all(x.shape == (self.N,) for x in vs)
        ct = np.empty((2, level + 1, self.N), dtype=np.uint64)
        self.L.orc_encrypt_noise(self._h, _p(np.ascontiguousarray(pk, dtype=np.uint64)), _p(m), level,
                                 *(_p(x, I64P) for x in vs), _p(ct))
        return Ciphertext(ct, level, scale)

    def decrypt(self, ct: Ciphertext, sk: np.ndarray) -> np.ndarray:
        m = np.empty((ct.level + 1, self.N), dtype=np.uint64)
        self.L.orc_decrypt(self._h, _p(sk, I64P), _p(np.ascontiguousarray(ct.data)), ct.level, _p(m))
        return m

    def decrypt_decode(self, ct: Ciphertext, sk: np.ndarray) -> np.ndarray:
        return enc.decode(self.decrypt(ct, sk), ct.scale, self.qs(ct.level), self.N)

    # ------------------------------------------------------------ ops
    def add(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        assert a.level == b.level
        out = np.empty_like(a.data)
        self.L.orc_add(self._h, _p(a.data), _p(b.data), a.level, _p(out))
        return Ciphertext(out, a.level, a.scale)

    def add_plain(self, a: Ciphertext, pt: np.ndarray) -> Ciphertext:
        out = np.empty_like(a.data)
        self.L.orc_add_plain(self._h, _p(a.data), _p(np.ascontiguousarray(pt)), a.level, _p(out))
        return Ciphertext(out, a.level, a.scale)

    def mult_plain(self, a: Ciphertext, pt: np.ndarray, pt_scale: float) -> Ciphertext:
        out = np.empty_like(a.data)
        self.L.orc_mult_plain(self._h, _p(a.data), _p(np.ascontiguousarray(pt)), a.level, _p(out))
        return Ciphertext(out, a.level, a.scale * pt_scale)

    def rescale(self, a: Ciphertext) -> Ciphertext:
        if a.level == 0:
            raise ValueError("rescale at level 0")
        out = np.empty((2, a.level, self.N), dtype=np.uint64)
        self.L.orc_rescale(self._h, _p(a.data), a.level, _p(out))
        return Ciphertext(out, a.level - 1, a.scale / self.pr.q[a.level])

    def modup(self, x: np.ndarray, level: int, digit: int) -> np.ndarray:
        out = np.empty((level + 1 + self.pr.K, self.N), dtype=np.uint64)
        self.L.orc_modup(self._h, _p(np.ascontiguousarray(x)), level, digit, _p(out))
        return out

    def moddown(self, y: np.ndarray, level: int) -> np.ndarray:
        out = np.empty((level + 1, self.N), dtype=np.uint64)
        self.L.orc_moddown(self._h, _p(np.ascontiguousarray(y)), level, _p(out))
        return out

    def keyswitch(self, d: np.ndarray, level: int, ksk: np.ndarray) -> np.ndarray:
        out = np.empty((2, level + 1, self.N), dtype=np.uint64)
        self.L.orc_keyswitch(self._h, _p(np.ascontiguousarray(d)), level, _p(ksk), _p(out))
        return out

    def rotate(self, a: Ciphertext, r: int, keys: Keys) -> Ciphertext:
        out = np.empty_like(a.data)
        key = keys.rot.get(int(r))
        if key is None and self.galois(r) != 1:
            raise KeyError(f"no rotation key for step {r}")
        kp = _p(key) if key is not None else _p(out)
        self.L.orc_rotate(self._h, _p(a.data), a.level, int(r), kp, _p(out))
        return Ciphertext(out, a.level, a.scale)

    def rotate_ext(self, a: Ciphertext, r: int, keys: Keys) -> np.ndarray:
        """rho^r(a) kept over Q_l u P (no ModDown): uint64 [2][l+1+K][N]."""
        out = np.empty((2, a.level + 1 + self.pr.K, self.N), dtype=np.uint64)
        key = keys.rot.get(int(r))
        if key is None and self.galois(r) != 1:
            raise KeyError(f"no rotation key for step {r}")
        kp = _p(key) if key is not None else None
        self.L.orc_rotate_ext(self._h, _p(a.data), a.level, int(r), kp, _p(out))
        return out

    def square(self, a: Ciphertext, keys: Keys) -> Ciphertext:
        out = np.empty_like(a.data)
        self.L.orc_square(self._h, _p(a.data), a.level, _p(keys.rlk), _p(out))
        return Ciphertext(out, a.level, a.scale * a.scale)

    def automorph(self, x: np.ndarray, g: int, prime_idx) -> np.ndarray:
        x = np.ascontiguousarray(x)
        out = np.empty_like(x)
        idx = np.asarray(prime_idx, dtype=np.int32)
        self.L.orc_automorph(self._h, len(idx), _p(idx, I32P), g, _p(x), _p(out))
        return out

    def polymul(self, a: np.ndarray, b: np.ndarray, prime_idx) -> np.ndarray:
        out = np.empty_like(a)
        idx = np.asarray(prime_idx, dtype=np.int32)
        self.L.orc_polymul(self._h, len(idx), _p(idx, I32P), _p(np.ascontiguousarray(a)),
                           _p(np.ascontiguousarray(b)), _p(out))
        return out

    def dense(self, a: Ciphertext, layer: "DenseLayer", keys: Keys) -> Ciphertext:
        if layer.level != a.level:
            raise ValueError("plaintexts encoded for another level")
        steps = sorted(keys.rot)
        step_arr = np.array(steps, dtype=np.int64)
        key_ptrs = (U64P * max(1, len(steps)))(*[_p(keys.rot[s]) for s in steps])
        out = np.empty_like(a.data)
        bias = _p(layer.bias) if layer.bias is not None else None
        rc = self.L.orc_dense_ex(self._h, _p(a.data), a.level, layer.m, layer.n, layer.n1, _p(layer.pts), bias,
                                 len(steps), _p(step_arr, I64P), key_ptrs, int(layer.qp), int(layer.rs_bits), _p(out))
        if rc != 0:
            raise RuntimeError(f"orc_dense failed ({rc})")
        return Ciphertext(out, a.level, a.scale * layer.pt_scale)

    def linear(self, cts: list, pts: np.ndarray, baby, giant, pt_scale: float, keys: Keys, only=None) -> list:
        """Multi-input linear transform in baby-step/giant-step form (the
        multi-channel convolution of oracle/conv.py):
            out[j] = sum_g rho^{giant[g]}( sum_{i,b} MultPlain(rho^{baby[b]}(cts[i]), pts[g][j][i][b]) ),
        giant[0] = 0; the sums over g accumulate in increasing g.  only: the
        output indices to compute (default all)."""
        n_giant, n_out, n_in, n_baby = pts.shape[:4]
        rot = [[self.rotate(ct, r, keys) for r in baby] for ct in cts]
        outs = []
        for j in (range(n_out) if only is None else only):
            z = None
            for g in range(n_giant):
                s = None
                for i in range(n_in):
                    for b in range(n_baby):
                        p = self.mult_plain(rot[i][b], pts[g, j, i, b], pt_scale)
                        s = p if s is None else self.add(s, p)
                if g == 0:
                    z = s
                else:
                    z = self.add(z, self.rotate(s, giant[g], keys))
            outs.append(z)
        return outs

    # ----------------------------------------------------------- network
    def prepare_dense(self, W: np.ndarray, b: np.ndarray | None, n1: int, level: int, in_scale: float,
                      pt_scale: float | None = None, qp: bool = False, rs_bits: int = 0) -> "DenseLayer":
        """Encode the pre-rotated diagonals (scale Delta_w, limbs q_0..q_l only:
        level-aware encoding; with qp, also p_0..p_{K-1} for the lazy-ModDown
        form) and the bias (scale in_scale * Delta_w, period m, limbs q_0..q_l)."""
        pr = self.pr
        pt_scale = pr.scale if pt_scale is None else pt_scale
        m, n = W.shape
        slots = planmod.plaintext_slots(W, n1, pr.slots)
        primes = self.qs(level) + (list(pr.p) if qp else [])
        pts = np.stack([enc.encode(slots[k], pt_scale, primes, self.N) for k in range(m)])
        bias = None
        if b is not None:
            bias = self.encode(planmod.bias_slots(b, pr.slots), in_scale * pt_scale, level)
        return DenseLayer(m, n, n1, level, pts, bias, pt_scale, in_scale * pt_scale, qp, rs_bits)

    def prepare_network(self, weights, biases, n1s, level=None, in_scale=None, qps=None, rs_bits=None) -> list:
        """Walk levels and scales: dense -> rescale -> (square -> rescale) ..."""
        pr = self.pr
        level = pr.L if level is None else level
        scale = pr.scale if in_scale is None else in_scale
        layers = []
        for li, (W, b, n1) in enumerate(zip(weights, biases, n1s)):
            lay = self.prepare_dense(W, b, n1, level, scale, qp=bool(qps[li]) if qps else False,
                                     rs_bits=int(rs_bits[li]) if rs_bits else 0)
            layers.append(lay)
            scale = scale * lay.pt_scale
            scale = scale / pr.q[level]
            level -= 1
            if li + 1 < len(weights):
                scale = scale * scale
                scale = scale / pr.q[level]
                level -= 1
        return layers

    def eval_network(self, ct: Ciphertext, layers: list, keys: Keys, progress=None) -> Ciphertext:
        """progress: optional callable(layer index) after each layer (long runs
        report that they are alive)."""
        for li, lay in enumerate(layers):
            ct = self.rescale(self.dense(ct, lay, keys))
            if li + 1 < len(layers):
                ct = self.rescale(self.square(ct, keys))
            if progress is not None:
                progress(li)
        return ct


@dataclass
class DenseLayer:
    m: int
    n: int
    n1: int
    level: int
    pts: np.ndarray            # uint64 [m][level+1(+K)][N], coefficient form, pre-rotated diagonals
    bias: np.ndarray | None    # uint64 [level+1][N]
    pt_scale: float
    bias_scale: float
    qp: bool = False           # diagonals over Q_l u P: lazy-ModDown evaluation (orc_dense_qp)
    rs_bits: int = 0           # rotate-and-sum: sequential (0) or hoisted groups of this many bits


def network_steps(layers_shape, rs_bits=None) -> list[int]:
    """Union of rotation steps of all dense layers [(m, n, n1), ...] (rs_bits:
    the rotate-and-sum form of each layer, default sequential)."""
    steps = set()
    for li, (m, n, n1) in enumerate(layers_shape):
        steps.update(planmod.rotation_steps(m, n, n1, rs_bits[li] if rs_bits else 0))
    return sorted(steps)

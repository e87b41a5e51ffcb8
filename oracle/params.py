"""Parameter presets and the prime-selection rule (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper fixes no CKKS parameters: it states only that they give 128-bit
security and that the RNS variant of CKKS in SEAL 3.4 was used (Methods,
"Experimental setting").  The presets below follow the workload
configurations of this project; the prime rule is: for a bit size b list
2^b + 1 - k*2N for k = 1, 2, ... (all congruent to 1 mod 2N and below 2^b),
keep the primes in descending order, and hand them out in the order q_0,
q_1..q_L, p_0..p_{K-1}, skipping primes already taken.
"""
from __future__ import annotations

from dataclasses import dataclass, field

# Deterministic Miller-Rabin: these bases are exact for every n < 3.3e24.
_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def primes_below(bits: int, two_n: int, count: int, taken=()) -> list[int]:
    """The ``count`` largest primes 2^bits + 1 - k*2N (k >= 1) not in ``taken``."""
    out, k = [], 1
    taken = set(taken)
    while len(out) < count:
        c = (1 << bits) + 1 - k * two_n
        if c < 2:
            raise ValueError("ran out of candidates")
        if c not in taken and is_prime(c):
            out.append(c)
        k += 1
    return out


def prime_chain(log_n: int, q_bits: list[int], p_bits: list[int]) -> tuple[list[int], list[int]]:
    """Primes for q_0..q_L (bit sizes q_bits) then p_0..p_{K-1} (p_bits)."""
    two_n = 2 << log_n
    taken: list[int] = []
    qs, ps = [], []
    for b in q_bits:
        qs.append(primes_below(b, two_n, 1, taken)[0])
        taken.append(qs[-1])
    for b in p_bits:
        ps.append(primes_below(b, two_n, 1, taken)[0])
        taken.append(ps[-1])
    return qs, ps


@dataclass
class Params:
    log_n: int
    q: list[int]
    p: list[int]
    alpha: int                  # primes per decomposition digit
    scale_bits: int             # Delta = 2^scale_bits (inputs and weights)
    name: str = ""
    sigma_w: float = 0.05       # weight / bias standard deviation
    layers: list[tuple[int, int, int]] = field(default_factory=list)  # (m, n, n1) per dense layer

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def slots(self) -> int:
        return self.n // 2

    @property
    def L(self) -> int:
        return len(self.q) - 1

    @property
    def K(self) -> int:
        return len(self.p)

    @property
    def dnum(self) -> int:
        return -(-len(self.q) // self.alpha)

    @property
    def scale(self) -> float:
        return float(2 ** self.scale_bits)


def make(log_n, q_bits, p_bits, alpha, scale_bits, name="", sigma_w=0.05, layers=()):
    q, p = prime_chain(log_n, q_bits, p_bits)
    return Params(log_n, q, p, alpha, scale_bits, name, sigma_w, list(layers))


def preset(name: str) -> Params:
    """Workload presets.

    cfg1  plain request: N=2^13, q0 45b, 3x35b, P 45b, alpha=1 (dnum=4); net 256->64, x^2, 64->2.
    cfg2  kernel micro-bench: N=2^16, 24 x 50b Q-limbs, 8 x 50b P-limbs, alpha=8 (dnum=3).
    cfg3  small net: N=2^15, q0 60b, 6x40b, P 2x60b, alpha=2 (dnum=4); 1024->128, x^2, 128->2.
    cfg4  large net: N=2^16, q0 60b, 10x45b, P 3x60b, alpha=3 (dnum=4); 4096->256->64->2.
    """
    if name == "cfg1":
        return make(13, [45] + [35] * 3, [45], 1, 35, name, 0.05, [(64, 256, 8), (2, 64, 2)])
    if name == "cfg2":
        return make(16, [50] * 24, [50] * 8, 8, 50, name)
    if name == "cfg3":
        return make(15, [60] + [40] * 6, [60] * 2, 2, 40, name, 0.03, [(128, 1024, 32), (2, 128, 2)])
    if name == "cfg4":
        return make(16, [60] + [45] * 10, [60] * 3, 3, 45, name, 0.02,
                    [(256, 4096, 16), (64, 256, 8), (2, 64, 2)])
    raise KeyError(name)


def tiny(log_n: int, n_q: int = 4, n_p: int = 2, alpha: int = 2, q_bits: int = 40, q0_bits: int = 50,
         p_bits: int = 50, scale_bits: int = 30) -> Params:
    """Small parameter sets for bit-exact cross-checks and fast parity tests."""
    return make(log_n, [q0_bits] + [q_bits] * (n_q - 1), [p_bits] * n_p, alpha, scale_bits, f"tiny{log_n}")

"""Independent pure-Python big-integer oracle for ring dimension N <= 64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A second, deliberately different implementation of every client and server
operation, used to cross-check the C++ oracle bit for bit at tiny N:
  * polynomial products are schoolbook negacyclic convolutions (no NTT);
  * fast base conversion (ModUp) and ModDown are evaluated as the exact
    integer sums they are defined by, then reduced, instead of limb by limb;
  * rescale is the exact integer division (c - [c]_{q_l}) / q_l of the CRT
    lift of each coefficient.
The sampling conventions (SplitMix64 sub-seeds, rejection rules, seed tags)
are restated here from their definitions, not imported.
"""
from __future__ import annotations

import math

MASK = (1 << 64) - 1

# Seed tags of the sampled client objects (same convention as the C++ core).
TAG_SECRET, TAG_PUBLIC, TAG_RELIN = 0x5EC, 0x9B, 0x4E1


def tag_rotation(r: int) -> int:
    return (0x40 << 32) | (r & 0xFFFFFFFF)


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014)."""

    def __init__(self, seed: int):
        self.s = seed & MASK

    def next(self) -> int:
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)


def derive_seed(master: int, tag: int) -> int:
    return SplitMix64(master ^ tag).next()


def sample_ternary(seed: int, n: int) -> list[int]:
    g = SplitMix64(seed)
    out = []
    while len(out) < n:
        v = g.next() & 3
        if v != 3:
            out.append(v - 1)
    return out


def sample_gaussian(seed: int, n: int) -> list[int]:
    g = SplitMix64(seed)
    out = []
    while len(out) < n:
        u1 = ((g.next() >> 11) + 1) * 2.0 ** -53
        u2 = (g.next() >> 11) * 2.0 ** -53
        x = math.sqrt(-2.0 * math.log(u1)) * math.cos(6.283185307179586476925286766559 * u2) * 3.2
        r = -math.floor(-x + 0.5) if x < 0 else math.floor(x + 0.5)
        if abs(r) <= 19:
            out.append(int(r))
    return out


def sample_uniform(seed: int, primes: list[int], n: int) -> list[list[int]]:
    g = SplitMix64(seed)
    out = []
    for q in primes:
        lim = ((1 << 64) // q) * q
        row = []
        while len(row) < n:
            w = g.next()
            if w < lim:
                row.append(w % q)
        out.append(row)
    return out


def negacyclic_mul(a: list[int], b: list[int], q: int) -> list[int]:
    """Schoolbook product modulo X^N + 1 and q."""
    n = len(a)
    c = [0] * n
    for i in range(n):
        if a[i] == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += a[i] * b[j]
            else:
                c[k - n] -= a[i] * b[j]
    return [v % q for v in c]


def automorph(a: list[int], g: int, q: int) -> list[int]:
    """a(X) -> a(X^g): X^(j g) = (-1)^floor(j g / N) X^(j g mod N)."""
    n = len(a)
    out = [0] * n
    for j in range(n):
        e = j * g
        sign = -1 if (e // n) % 2 else 1
        out[e % n] = (sign * a[j]) % q
    return out


class Tiny:
    def __init__(self, n: int, q: list[int], p: list[int], alpha: int):
        assert n <= 64
        self.n, self.q, self.p, self.alpha = n, list(q), list(p), alpha
        self.all = self.q + self.p

    # --------------------------------------------------------- client
    def dnum(self):
        return -(-len(self.q) // self.alpha)

    def secret(self, seed):
        return sample_ternary(derive_seed(seed, TAG_SECRET), self.n)

    def _ext(self, level):
        return self.q[: level + 1] + self.p

    def public_key(self, s, seed):
        a = sample_uniform(derive_seed(seed, 0x11), self.q, self.n)
        e = sample_gaussian(derive_seed(seed, 0x12), self.n)
        b = [[(-x + y) % q for x, y in zip(negacyclic_mul(a[i], s, q), e)] for i, q in enumerate(self.q)]
        return [b, a]

    def switch_key(self, s, s_prime_int, seed):
        """s_prime_int: integer coefficients of the target secret."""
        P = 1
        for pk in self.p:
            P *= pk
        keys = []
        for j in range(self.dnum()):
            a = sample_uniform(derive_seed(seed, 0x100 + 2 * j), self.all, self.n)
            e = sample_gaussian(derive_seed(seed, 0x101 + 2 * j), self.n)
            b = []
            for i, q in enumerate(self.all):
                row = [(-x + y) % q for x, y in zip(negacyclic_mul(a[i], s, q), e)]
                if i < len(self.q) and i // self.alpha == j:
                    row = [(v + P * sp) % q for v, sp in zip(row, s_prime_int)]
                b.append(row)
            keys.append([b, a])
        return keys

    def keygen(self, seed, steps=(), relin=True):
        s = self.secret(seed)
        pk = self.public_key(s, derive_seed(seed, TAG_PUBLIC))
        rlk = None
        if relin:
            s2 = negacyclic_mul(s, s, 1 << 200)               # exact integer square (no wrap at this modulus)
            s2 = [v - (1 << 200) if v >= 1 << 199 else v for v in s2]
            rlk = self.switch_key(s, s2, derive_seed(seed, TAG_RELIN))
        rot = {}
        for r in steps:
            g = self.galois(r)
            sg = automorph(s, g, 1 << 200)
            sg = [v - (1 << 200) if v >= 1 << 199 else v for v in sg]
            rot[int(r)] = self.switch_key(s, sg, derive_seed(seed, tag_rotation(int(r))))
        return s, pk, rlk, rot

    def encrypt(self, m, pk, seed):
        v = sample_ternary(derive_seed(seed, 0x21), self.n)
        e0 = sample_gaussian(derive_seed(seed, 0x22), self.n)
        e1 = sample_gaussian(derive_seed(seed, 0x23), self.n)
        c0, c1 = [], []
        for i, q in enumerate(self.q):
            vb = negacyclic_mul(v, pk[0][i], q)
            va = negacyclic_mul(v, pk[1][i], q)
            c0.append([(x + e + mm) % q for x, e, mm in zip(vb, e0, m[i])])
            c1.append([(x + e) % q for x, e in zip(va, e1)])
        return [c0, c1]

    def decrypt(self, ct, s, level):
        return [[(x + y) % q for x, y in zip(ct[0][i], negacyclic_mul(ct[1][i], s, q))]
                for i, q in enumerate(self.q[: level + 1])]

    # --------------------------------------------------------- server
    def galois(self, r):
        return pow(5, r % (self.n // 2), 2 * self.n)

    def add(self, a, b, level):
        return [[[(x + y) % q for x, y in zip(a[k][i], b[k][i])] for i, q in enumerate(self.q[: level + 1])]
                for k in range(2)]

    def mult_plain(self, ct, pt, level):
        return [[negacyclic_mul(ct[k][i], pt[i], q) for i, q in enumerate(self.q[: level + 1])] for k in range(2)]

    def add_plain(self, ct, pt, level):
        return [[[(x + y) % q for x, y in zip(ct[0][i], pt[i])] for i, q in enumerate(self.q[: level + 1])],
                [row[:] for row in ct[1]]]

    def _crt(self, res, mods):
        M = 1
        for m in mods:
            M *= m
        out = []
        for k in range(self.n):
            x = 0
            for r, m in zip(res, mods):
                mh = M // m
                x += r[k] * mh * pow(mh, -1, m)
            out.append(x % M)
        return out, M

    def rescale(self, ct, level):
        mods = self.q[: level + 1]
        ql = mods[-1]
        out = []
        for poly in ct:
            lift, _ = self._crt(poly, mods)
            exact = [(x - x % ql) // ql for x in lift]               # exact division
            out.append([[v % q for v in exact] for q in mods[:-1]])
        return out

    def modup(self, x, level, digit):
        """Conv(x) as the exact integer sum_i [x_i (Q_D/q_i)^-1]_{q_i} (Q_D/q_i), reduced."""
        D = list(range(digit * self.alpha, min((digit + 1) * self.alpha, level + 1)))
        QD = 1
        for i in D:
            QD *= self.q[i]
        big = [0] * self.n
        for i in D:
            qi = self.q[i]
            hat = QD // qi
            hinv = pow(hat % qi, -1, qi)
            for k in range(self.n):
                big[k] += (x[i][k] * hinv % qi) * hat
        out = []
        for t, mod in enumerate(self._ext(level)):
            out.append(list(x[t]) if t in D else [v % mod for v in big])
        return out

    def moddown(self, y, level):
        P = 1
        for pk in self.p:
            P *= pk
        big = [0] * self.n
        for k_, pk in enumerate(self.p):
            hat = P // pk
            hinv = pow(hat % pk, -1, pk)
            row = y[level + 1 + k_]
            for k in range(self.n):
                big[k] += (row[k] * hinv % pk) * hat
        out = []
        for i, q in enumerate(self.q[: level + 1]):
            pinv = pow(P % q, -1, q)
            out.append([((y[i][k] - big[k]) * pinv) % q for k in range(self.n)])
        return out

    def _ks_ext(self, d, level, ksk, g):
        """Key-switch inner product over Q_l u P, before ModDown."""
        ext_mods = self._ext(level)
        ext_idx = list(range(level + 1)) + [len(self.q) + k for k in range(len(self.p))]
        ub = [[0] * self.n for _ in ext_mods]
        ua = [[0] * self.n for _ in ext_mods]
        for j in range(-(-(level + 1) // self.alpha)):
            ext = self.modup(d, level, j)
            if g != 1:
                ext = [automorph(row, g, m) for row, m in zip(ext, ext_mods)]
            for t, (m, ki) in enumerate(zip(ext_mods, ext_idx)):
                pb = negacyclic_mul(ext[t], ksk[j][0][ki], m)
                pa = negacyclic_mul(ext[t], ksk[j][1][ki], m)
                ub[t] = [(x + y) % m for x, y in zip(ub[t], pb)]
                ua[t] = [(x + y) % m for x, y in zip(ua[t], pa)]
        return ub, ua

    def _ks(self, d, level, ksk, g):
        ub, ua = self._ks_ext(d, level, ksk, g)
        return [self.moddown(ub, level), self.moddown(ua, level)]

    def keyswitch(self, d, level, ksk):
        return self._ks(d, level, ksk, 1)

    def rotate(self, ct, level, r, rot):
        g = self.galois(r)
        if g == 1:
            return [[row[:] for row in p] for p in ct]
        ks = self._ks(ct[1], level, rot[int(r)], g)
        c0 = [automorph(row, g, q) for row, q in zip(ct[0], self.q[: level + 1])]
        return [[[(x + y) % q for x, y in zip(c0[i], ks[0][i])] for i, q in enumerate(self.q[: level + 1])], ks[1]]

    def square(self, ct, level, rlk):
        mods = self.q[: level + 1]
        d0 = [negacyclic_mul(ct[0][i], ct[0][i], q) for i, q in enumerate(mods)]
        d1 = [[2 * v % q for v in negacyclic_mul(ct[0][i], ct[1][i], q)] for i, q in enumerate(mods)]
        d2 = [negacyclic_mul(ct[1][i], ct[1][i], q) for i, q in enumerate(mods)]
        ks = self._ks(d2, level, rlk, 1)
        return [[[(x + y) % q for x, y in zip(d0[i], ks[0][i])] for i, q in enumerate(mods)],
                [[(x + y) % q for x, y in zip(d1[i], ks[1][i])] for i, q in enumerate(mods)]]

    def rotate_ext(self, ct, level, r, rot):
        """rho^r(ct) over Q_l u P without ModDown: (P sigma(c0) + u_b, u_a);
        P times anything vanishes modulo the p_k.  r = 0: (P c0, P c1)."""
        P = math.prod(self.p)
        mods = self.q[: level + 1]
        zeros = [[0] * self.n for _ in self.p]
        g = self.galois(r)
        if g == 1:
            return [[[v * P % q for v in ct[k][i]] for i, q in enumerate(mods)] + [row[:] for row in zeros]
                    for k in range(2)]
        ub, ua = self._ks_ext(ct[1], level, rot[int(r)], g)
        c0 = [automorph(row, g, q) for row, q in zip(ct[0], mods)]
        b = [[(x + v * P) % q for x, v in zip(ub[i], c0[i])] for i, q in enumerate(mods)] + ub[level + 1:]
        return [b, ua]

    def _rotate_sum_hoisted(self, z, level, m, n, bits, rot):
        """Hoisted rotate-and-sum: per group of b bits (most significant first)
        with base shift t, z <- ModDown(sum_{k < 2^b} rho_ext^{k t}(z))."""
        mods = self._ext(level)
        left = (n // m).bit_length() - 1
        while left > 0:
            b = min(bits, left)
            left -= b
            t = m << left
            acc = [[[0] * self.n for _ in mods] for _ in range(2)]
            for k in range(1 << b):
                r = self.rotate_ext(z, level, k * t, rot)
                for p in range(2):
                    for i, q in enumerate(mods):
                        acc[p][i] = [(x + y) % q for x, y in zip(acc[p][i], r[p][i])]
            z = [self.moddown(acc[0], level), self.moddown(acc[1], level)]
        return z

    def _dense_tail(self, sums, level, m, n, n1, bias, rot, rs_bits=0):
        z = sums[0]
        for j in range(1, len(sums)):
            z = self.add(z, self.rotate(sums[j], level, n1 * j, rot), level)
        if rs_bits > 0:
            z = self._rotate_sum_hoisted(z, level, m, n, rs_bits, rot)
        else:
            t = n // 2
            while t >= m:
                z = self.add(z, self.rotate(z, level, t, rot), level)
                t //= 2
        if bias is not None:
            z = self.add_plain(z, bias, level)
        return z

    def dense(self, ct, level, m, n, n1, pts, bias, rot, rs_bits=0):
        n2 = m // n1
        baby = [ct] + [self.rotate(ct, level, i, rot) for i in range(1, n1)]
        sums = []
        for j in range(n2):
            s = None
            for i in range(n1):
                prod = self.mult_plain(baby[i], pts[n1 * j + i], level)
                s = prod if s is None else self.add(s, prod, level)
            sums.append(s)
        return self._dense_tail(sums, level, m, n, n1, bias, rot, rs_bits)

    def dense_qp(self, ct, level, m, n, n1, pts, bias, rot, rs_bits=0):
        """Lazy-ModDown dense: inner sums over Q_l u P (pts over Q_l u P), one
        ModDown per inner sum, then the same giant steps / rotate-and-sum / bias."""
        n2 = m // n1
        mods = self._ext(level)
        baby = [self.rotate_ext(ct, level, i, rot) for i in range(n1)]
        sums = []
        for j in range(n2):
            acc = [[[0] * self.n for _ in mods] for _ in range(2)]
            for i in range(n1):
                pt = pts[n1 * j + i]
                for k in range(2):
                    for t, q in enumerate(mods):
                        pr = negacyclic_mul(baby[i][k][t], pt[t], q)
                        acc[k][t] = [(x + y) % q for x, y in zip(acc[k][t], pr)]
            sums.append([self.moddown(acc[0], level), self.moddown(acc[1], level)])
        return self._dense_tail(sums, level, m, n, n1, bias, rot, rs_bits)

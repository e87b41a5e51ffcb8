"""Pins of the CPU oracle against mathematics it must satisfy (no GPU).

Each test checks the oracle against something other than itself: hand-worked
closed forms (tests/golden), schoolbook products, evaluation at roots of
X^N + 1, exact big-integer identities of the RNS base conversions and of
rescaling, decryption correctness, slot-level identities of rotation and
square, the FP64 plaintext network, and the independent big-integer twin
oracle/tiny.py.
"""
import json
import os

import numpy as np
import pytest

from oracle import ckks, encode as enc, params, plainnet, plan, tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_params(log_n=10, nq=4, np_=2, alpha=2):
    return params.make(log_n, [50] + [35] * (nq - 1), [50] * np_, alpha, 35)


@pytest.fixture(scope="module")
def o10(oracle_lib):
    return ckks.Oracle(small_params())


@pytest.fixture(scope="module")
def keys10(o10):
    return o10.keygen(11, steps=[1, 2, 3, 5, 7, 8, 16, 64, 256, -1])


# ------------------------------------------------------------------ primes
@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3", "cfg4"])
def test_prime_chain_properties(name):
    pr = params.preset(name)
    allp = pr.q + pr.p
    assert len(set(allp)) == len(allp)
    for q in allp:
        assert params.is_prime(q) and q % (2 * pr.n) == 1 and q < 2 ** 61
    bits = {"cfg1": ([45, 35, 35, 35], [45]), "cfg3": ([60] + [40] * 6, [60, 60]),
            "cfg4": ([60] + [45] * 10, [60] * 3), "cfg2": ([50] * 24, [50] * 8)}[name]
    assert [q.bit_length() for q in pr.q] == bits[0]
    assert [p.bit_length() for p in pr.p] == bits[1]


def test_prime_rule_brute_force():
    # Largest primes below 2^20 that are 1 mod 2N (N = 2^6), by trial division.
    two_n = 128
    brute = [c for c in range(2 ** 20 - 1, 0, -1) if c % two_n == 1 and all(c % d for d in range(2, int(c ** 0.5) + 1))][:3]
    assert params.primes_below(20, two_n, 3) == brute
    qs, ps = params.prime_chain(6, [20, 20], [20])
    assert qs + ps == brute


def test_miller_rabin_against_sieve():
    lim = 20000
    sieve = np.ones(lim, bool)
    sieve[:2] = False
    for i in range(2, int(lim ** 0.5) + 1):
        sieve[i * i::i] = False
    assert all(params.is_prime(i) == bool(sieve[i]) for i in range(lim))
    assert not params.is_prime(3215031751)           # strong pseudoprime to bases 2, 3, 5, 7


# ------------------------------------------------------ ring arithmetic
def test_golden_negacyclic_n4():
    g = json.load(open(os.path.join(GOLDEN, "negacyclic_n4_q17.json")))
    for c in g["cases"]:
        assert tiny.negacyclic_mul(c["a"], c["b"], g["q"]) == c["product"]


@pytest.mark.parametrize("log_n", [4, 5, 6])
def test_polymul_matches_schoolbook(oracle_lib, log_n):
    pr = params.make(log_n, [50, 40, 40], [50], 1, 30)
    o = ckks.Oracle(pr)
    rng = np.random.default_rng(log_n)
    for i, q in enumerate(pr.q + pr.p):
        a = rng.integers(0, q, pr.n, dtype=np.uint64)
        b = rng.integers(0, q, pr.n, dtype=np.uint64)
        got = o.polymul(a[None], b[None], [i])[0]
        assert got.tolist() == tiny.negacyclic_mul(a.tolist(), b.tolist(), q)


def horner(coeffs, x, q):
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * x + c) % q
    return acc


@pytest.mark.parametrize("log_n", [13, 16])
def test_polymul_at_roots_large_n(oracle_lib, log_n):
    pr = params.make(log_n, [60], [], 1, 30)
    o = ckks.Oracle(pr)
    q, n = pr.q[0], pr.n
    psi = o.psi(0)
    assert pow(psi, n, q) == q - 1                     # psi has order exactly 2N
    rng = np.random.default_rng(5)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    c = o.polymul(a[None], b[None], [0])[0]
    for t in (1, 2 * int(rng.integers(0, n)) + 1):
        x = pow(psi, t, q)                             # a root of X^N + 1
        assert horner(c.tolist(), x, q) == horner(a.tolist(), x, q) * horner(b.tolist(), x, q) % q


def test_golden_slot_rotation_n8():
    g = json.load(open(os.path.join(GOLDEN, "slot_rotation_n8.json")))
    assert enc.slot_exponents(g["n"]).tolist() == g["slot_exponents"]
    t = tiny.Tiny(g["n"], [17], [], 1)
    for r, ge in g["galois_left_rotation"].items():
        assert t.galois(int(r)) == ge
    q = 97
    for case in g["automorph_g5"]:
        assert tiny.automorph(case["in"], 5, q) == [v % q for v in case["out_signed"]]


def test_automorphism_identities(o10):
    n = o10.N
    q = o10.pr.q[0]
    psi = o10.psi(0)
    rng = np.random.default_rng(3)
    a = rng.integers(0, q, n, dtype=np.uint64)
    for g in (5, 25, 2 * n - 1, o10.galois(7)):
        sa = o10.automorph(a[None], g, [0])[0]
        x = pow(psi, 2 * int(rng.integers(0, n)) + 1, q)
        assert horner(sa.tolist(), x, q) == horner(a.tolist(), pow(x, g, q), q)
    g, h = o10.galois(3), o10.galois(5)
    comp = o10.automorph(o10.automorph(a[None], h, [0]), g, [0])[0]
    assert np.array_equal(comp, o10.automorph(a[None], g * h % (2 * n), [0])[0])
    assert o10.galois(3) * o10.galois(5) % (2 * n) == o10.galois(8)
    order = next(k for k in range(1, n + 1) if pow(5, k, 2 * n) == 1)
    assert order == n // 2
    assert o10.galois(-1) == o10.galois(n // 2 - 1)


def test_automorph_c_matches_tiny(oracle_lib):
    pr = params.make(6, [40], [], 1, 30)
    o = ckks.Oracle(pr)
    a = np.random.default_rng(0).integers(0, pr.q[0], pr.n, dtype=np.uint64)
    for g in (5, 25, 127, 3):
        assert o.automorph(a[None], g, [0])[0].tolist() == tiny.automorph(a.tolist(), g, pr.q[0])


# ------------------------------------------------------- encode / decode
def test_encode_constant_vector():
    n = 1024
    c = 0.3125
    M = enc.encode_coeffs(np.full(n // 2, c), 2.0 ** 30, n)
    assert M[0] == round(c * 2 ** 30)
    assert np.all(np.abs(M[1:]) <= 1)


def test_encode_fft_equals_direct():
    n = 256
    z = np.random.default_rng(1).uniform(-1, 1, n // 2) + 0j
    a = enc.encode_coeffs(z, 2.0 ** 35, n)
    b = enc.encode_coeffs(z, 2.0 ** 35, n, direct=True)
    assert np.max(np.abs(a - b)) <= 1


def test_decode_inverts_encode():
    n = 2048
    z = np.random.default_rng(2).uniform(-1, 1, n // 2)
    primes = params.prime_chain(11, [50, 40], [])[0]
    res = enc.encode(z, 2.0 ** 40, primes, n)
    back = enc.decode(res, 2.0 ** 40, primes, n)
    assert np.max(np.abs(back - z)) < 2.0 ** -25


def test_encode_rotation_is_automorphism():
    n = 512
    z = np.random.default_rng(4).uniform(-1, 1, n // 2)
    r = 37
    Mz = enc.encode_coeffs(z, 2.0 ** 30, n).astype(np.int64)
    Mr = enc.encode_coeffs(np.roll(z, -r), 2.0 ** 30, n).astype(np.int64)
    g = pow(5, r, 2 * n)
    big = 1 << 62                                       # exact signed automorphism via a huge modulus
    sig = np.array(tiny.automorph([int(v) % big for v in Mz], g, big), dtype=object)
    sig = np.array([v - big if v >= big // 2 else v for v in sig], dtype=np.int64)
    assert np.max(np.abs(sig - Mr)) <= 1


# ----------------------------------------------------- base conversions
def crt(rows, mods):
    M = 1
    for m in mods:
        M *= m
    out = []
    for k in range(len(rows[0])):
        x = 0
        for r, m in zip(rows, mods):
            h = M // m
            x += int(r[k]) * h * pow(h % m, -1, m)
        out.append(x % M)
    return out, M


def test_modup_bigint_identity(oracle_lib):
    pr = params.make(6, [50, 40, 40, 40, 40], [50, 50, 50], 3, 30)
    o = ckks.Oracle(pr)
    rng = np.random.default_rng(8)
    level = 4
    x = np.stack([rng.integers(0, q, pr.n, dtype=np.uint64) for q in pr.q[: level + 1]])
    ext_mods = pr.q[: level + 1] + pr.p
    for digit in range(2):
        D = list(range(digit * 3, min(digit * 3 + 3, level + 1)))
        y = o.modup(x, level, digit)
        X, QD = crt([x[i] for i in D], [pr.q[i] for i in D])
        for k in range(pr.n):
            us = set()
            for t, m in enumerate(ext_mods):
                if t in D:
                    assert int(y[t][k]) == int(x[t][k])
                    continue
                u = (int(y[t][k]) - X[k]) * pow(QD % m, -1, m) % m
                us.add(u)
            assert len(us) == 1 and 0 <= us.pop() < len(D)


def test_moddown_bigint_identity(oracle_lib):
    pr = params.make(6, [50, 40, 40], [50, 50, 50], 3, 30)
    o = ckks.Oracle(pr)
    rng = np.random.default_rng(9)
    level = 2
    mods = pr.q[: level + 1] + pr.p
    y = np.stack([rng.integers(0, m, pr.n, dtype=np.uint64) for m in mods])
    out = o.moddown(y, level)
    Y, _ = crt(list(y), mods)
    P = 1
    for p in pr.p:
        P *= p
    for k in range(pr.n):
        yP = Y[k] % P
        base = (Y[k] - yP) // P
        vs = {(base - int(out[i][k])) % q for i, q in enumerate(pr.q[: level + 1])}
        assert len(vs) == 1 and 0 <= vs.pop() < len(pr.p)


def test_rescale_bigint_exact(o10):
    pr = o10.pr
    rng = np.random.default_rng(10)
    level = 3
    data = np.stack([np.stack([rng.integers(0, q, pr.n, dtype=np.uint64) for q in pr.q[: level + 1]])
                     for _ in range(2)])
    out = o10.rescale(ckks.Ciphertext(data, level, 2.0 ** 70))
    ql = pr.q[level]
    for p in range(2):
        C, _ = crt(list(data[p]), pr.q[: level + 1])
        for k in range(0, pr.n, 7):
            exact = (C[k] - C[k] % ql) // ql
            assert [int(out.data[p][i][k]) for i in range(level)] == [exact % q for q in pr.q[:level]]
    assert out.scale == 2.0 ** 70 / ql and out.level == level - 1


# --------------------------------------------------- encryption-level
def test_encrypt_decrypt(o10, keys10):
    z = np.random.default_rng(12).uniform(-1, 1, o10.pr.slots)
    ct = o10.encrypt(z, keys10.pk, 77)
    assert np.max(np.abs(o10.decrypt_decode(ct, keys10.sk) - z)) < 2.0 ** -18


def test_keyswitch_relin_and_identity(o10, keys10):
    pr = o10.pr
    n = pr.n
    level = pr.L
    qs = pr.q[: level + 1]
    rng = np.random.default_rng(13)
    d = np.stack([rng.integers(0, q, n, dtype=np.uint64) for q in qs])
    s = keys10.sk
    s_rns = np.stack([np.mod(s, np.int64(q)).astype(np.uint64) for q in pr.q + pr.p])
    idx = list(range(level + 1))
    s_ident = o10.switch_key(s, s_rns, 4242)             # switch key from s to s
    s2 = o10.polymul(s_rns[: level + 1], s_rns[: level + 1], idx)
    for ksk, target in ((keys10.rlk, s2), (s_ident, s_rns[: level + 1])):
        ks = o10.keyswitch(d, level, ksk)
        dec = o10.polymul(ks[1], s_rns[: level + 1], idx)
        want = o10.polymul(d, target, idx)
        err = []
        for i, q in enumerate(qs):
            e = (dec[i].astype(object) + ks[0][i].astype(object) - want[i].astype(object)) % q
            err.append(np.array([int(v) - q if int(v) > q // 2 else int(v) for v in e]))
        err = np.array(err)
        assert np.all(err == err[0])                 # one small integer error polynomial over every limb
        assert np.max(np.abs(err[0])) < 2 ** 20


def test_rotation_slots(o10, keys10):
    z = np.random.default_rng(14).uniform(-1, 1, o10.pr.slots)
    ct = o10.encrypt(z, keys10.pk, 78)
    for r in (1, 3, 7, 256, -1):
        got = o10.decrypt_decode(o10.rotate(ct, r, keys10), keys10.sk).real
        assert np.max(np.abs(got - np.roll(z, -r))) < 2.0 ** -16
    two = o10.rotate(o10.rotate(ct, 3, keys10), 5, keys10)
    one = o10.rotate(ct, 8, keys10)
    assert np.max(np.abs(o10.decrypt_decode(two, keys10.sk) - o10.decrypt_decode(one, keys10.sk))) < 2.0 ** -15
    assert np.array_equal(o10.rotate(ct, 0, keys10).data, ct.data)


def test_square_slots(o10, keys10):
    z = np.random.default_rng(15).uniform(-1, 1, o10.pr.slots)
    ct = o10.encrypt(z, keys10.pk, 79)
    sq = o10.square(ct, keys10)
    assert sq.scale == ct.scale * ct.scale
    got = o10.decrypt_decode(o10.rescale(sq), keys10.sk).real
    assert np.max(np.abs(got - z * z)) < 2.0 ** -16


@pytest.mark.parametrize("m,n,n1", [(8, 64, 1), (8, 64, 2), (8, 64, 8), (4, 16, 2), (16, 16, 4)])
def test_dense_slots(o10, keys10, m, n, n1):
    pr = o10.pr
    rng = np.random.default_rng(m * 100 + n + n1)
    W = rng.normal(0, 0.1, (m, n))
    b = rng.normal(0, 0.1, m)
    x = rng.uniform(-1, 1, n)
    steps = plan.rotation_steps(m, n, n1)
    keys = o10.keygen(11, steps=steps) if not set(steps) <= set(keys10.rot) else keys10
    ct = o10.encrypt(plan.input_slots(x, pr.slots), keys.pk, 80)
    lay = o10.prepare_dense(W, b, n1, ct.level, ct.scale)
    out = o10.dense(ct, lay, keys)
    got = o10.decrypt_decode(o10.rescale(out), keys.sk).real
    want = plan.bias_slots(W @ x + b, pr.slots)
    assert np.max(np.abs(got - want)) < 2.0 ** -14


# ------------------------------------------ lazy-ModDown (double-hoisted) dense
@pytest.mark.parametrize("r", [0, 1, 3, -1])
def test_rotate_ext_moddown_is_rotate(o10, keys10, r):
    # ModDown(P sigma(c0) + u_b) = sigma(c0) + ModDown(u_b) exactly: the
    # extended baby step brought down equals the ordinary rotation bit for bit.
    z = np.random.default_rng(40 + r).uniform(-1, 1, o10.pr.slots)
    ct = o10.encrypt(z, keys10.pk, 90)
    ext = o10.rotate_ext(ct, r, keys10)
    L = ct.level
    assert ext.shape == (2, L + 1 + o10.pr.K, o10.N)
    assert not ext[:, L + 1:].any() if r == 0 else True
    down = np.stack([o10.moddown(ext[0], L), o10.moddown(ext[1], L)])
    assert np.array_equal(down, o10.rotate(ct, r, keys10).data)


def _unit_layer(o, level, m, n, n1, taps):
    """Diagonals over Q_l u P equal to the constant polynomial 1 at the listed
    indices and 0 elsewhere (no encoding involved)."""
    ne = level + 1 + o.pr.K
    pts = np.zeros((m, ne, o.N), dtype=np.uint64)
    for k in taps:
        pts[k, :, 0] = 1
    return ckks.DenseLayer(m, n, n1, level, pts, None, 1.0, 1.0, qp=True)


def test_dense_qp_unit_diagonals_exact(o10, keys10):
    # With 0/1 constant diagonals the P-limbs of every product are those of
    # the extended rotations themselves, so one ModDown per inner sum is the
    # sum of exact rotations: closed forms in terms of the ordinary rotate.
    z = np.random.default_rng(41).uniform(-1, 1, o10.pr.slots)
    ct = o10.encrypt(z, keys10.pk, 91)
    R1 = o10.rotate(ct, 1, keys10)
    got = o10.dense(ct, _unit_layer(o10, ct.level, 2, 2, 2, [1]), keys10)
    assert np.array_equal(got.data, R1.data)
    got = o10.dense(ct, _unit_layer(o10, ct.level, 2, 2, 2, [0, 1]), keys10)
    assert np.array_equal(got.data, o10.add(ct, R1).data)
    # two inner sums, both = rho^1(ct): z = s_0 + rho^2(s_1)
    got = o10.dense(ct, _unit_layer(o10, ct.level, 4, 4, 2, [1, 3]), keys10)
    assert np.array_equal(got.data, o10.add(R1, o10.rotate(R1, 2, keys10)).data)


@pytest.mark.parametrize("m,n", [(8, 64), (16, 16)])
def test_dense_qp_one_baby_step_equals_dense(o10, keys10, m, n):
    # n1 = 1: the only extended "rotation" is P ct, and ModDown(P x) = x
    # exactly, so the lazy form reproduces the ordinary dense layer bit for bit.
    rng = np.random.default_rng(42 + m)
    W, b, x = rng.normal(0, 0.1, (m, n)), rng.normal(0, 0.1, m), rng.uniform(-1, 1, n)
    steps = plan.rotation_steps(m, n, 1)
    keys = o10.keygen(11, steps=steps) if not set(steps) <= set(keys10.rot) else keys10
    ct = o10.encrypt(plan.input_slots(x, o10.pr.slots), keys.pk, 92)
    std = o10.dense(ct, o10.prepare_dense(W, b, 1, ct.level, ct.scale), keys)
    lazy = o10.dense(ct, o10.prepare_dense(W, b, 1, ct.level, ct.scale, qp=True), keys)
    assert np.array_equal(std.data, lazy.data)


@pytest.mark.parametrize("m,n,n1", [(8, 64, 2), (8, 64, 8), (16, 16, 4), (16, 64, 16)])
def test_dense_qp_slots(o10, keys10, m, n, n1):
    # General diagonals: the result decrypts to W x + b (FP64) and to the
    # ordinary dense layer's value within the rounding of one ModDown.
    pr = o10.pr
    rng = np.random.default_rng(m * 100 + n + n1 + 7)
    W, b, x = rng.normal(0, 0.1, (m, n)), rng.normal(0, 0.1, m), rng.uniform(-1, 1, n)
    steps = plan.rotation_steps(m, n, n1)
    keys = o10.keygen(11, steps=steps) if not set(steps) <= set(keys10.rot) else keys10
    ct = o10.encrypt(plan.input_slots(x, pr.slots), keys.pk, 93)
    lay = o10.prepare_dense(W, b, n1, ct.level, ct.scale, qp=True)
    assert lay.pts.shape == (m, ct.level + 1 + pr.K, pr.n)
    out = o10.dense(ct, lay, keys)
    got = o10.decrypt_decode(o10.rescale(out), keys.sk).real
    want = plan.bias_slots(W @ x + b, pr.slots)
    assert np.max(np.abs(got - want)) < 2.0 ** -14
    std = o10.dense(ct, o10.prepare_dense(W, b, n1, ct.level, ct.scale), keys)
    ref = o10.decrypt_decode(o10.rescale(std), keys.sk).real
    assert np.max(np.abs(got - ref)) < 2.0 ** -18
    if n1 > 1:
        assert not np.array_equal(out.data, std.data)   # a different rounding point


# ------------------------------------------------- hoisted rotate-and-sum
def _dense_case(o, keys0, m, n, n1, seed, qp=False, rs_bits=0, extra_rs=()):
    pr = o.pr
    rng = np.random.default_rng(seed)
    W, b, x = rng.normal(0, 0.1, (m, n)), rng.normal(0, 0.1, m), rng.uniform(-1, 1, n)
    steps = set(plan.rotation_steps(m, n, n1, rs_bits))
    for r in extra_rs:
        steps |= set(plan.rotation_steps(m, n, n1, r))
    keys = keys0 if steps <= set(keys0.rot) else o.keygen(11, steps=sorted(steps | set(keys0.rot)))
    ct = o.encrypt(plan.input_slots(x, pr.slots), keys.pk, seed + 7)
    return W, b, x, keys, ct


@pytest.mark.parametrize("m,n,n1,qp", [(4, 64, 2, False), (4, 64, 2, True), (2, 16, 1, False), (8, 256, 4, True)])
def test_rotate_sum_one_bit_groups_are_sequential(o10, keys10, m, n, n1, qp):
    # A hoisted group of one bit is ModDown(P z + rho_ext^t(z)) = z + rho^t(z)
    # exactly, and the groups run from the largest shift down, so rs_bits = 1
    # reproduces the sequential rotate-and-sum bit for bit.
    W, b, x, keys, ct = _dense_case(o10, keys10, m, n, n1, 50 + m + n, qp, 0, (1,))
    seq = o10.dense(ct, o10.prepare_dense(W, b, n1, ct.level, ct.scale, qp=qp), keys)
    one = o10.dense(ct, o10.prepare_dense(W, b, n1, ct.level, ct.scale, qp=qp, rs_bits=1), keys)
    assert np.array_equal(seq.data, one.data)


@pytest.mark.parametrize("m,n,n1,qp,rs_bits", [(4, 64, 2, False, 2), (4, 64, 2, True, 4), (2, 128, 2, False, 3),
                                               (8, 256, 4, True, 3), (16, 16, 4, False, 2)])
def test_rotate_sum_hoisted_slots(o10, keys10, m, n, n1, qp, rs_bits):
    # Groups of several bits: decrypts to W x + b and to the sequential form's
    # value within the rounding of the extra ModDowns (n = m: no rotate-and-sum,
    # identical to the sequential form).
    pr = o10.pr
    W, b, x, keys, ct = _dense_case(o10, keys10, m, n, n1, 60 + m + n, qp, rs_bits)
    hz = o10.dense(ct, o10.prepare_dense(W, b, n1, ct.level, ct.scale, qp=qp, rs_bits=rs_bits), keys)
    got = o10.decrypt_decode(o10.rescale(hz), keys.sk).real
    assert np.max(np.abs(got - plan.bias_slots(W @ x + b, pr.slots))) < 2.0 ** -14
    keys_s = keys if set(plan.rotation_steps(m, n, n1)) <= set(keys.rot) else \
        o10.keygen(11, steps=sorted(set(keys.rot) | set(plan.rotation_steps(m, n, n1))))
    seq = o10.dense(ct, o10.prepare_dense(W, b, n1, ct.level, ct.scale, qp=qp), keys_s)
    ref = o10.decrypt_decode(o10.rescale(seq), keys.sk).real
    assert np.max(np.abs(got - ref)) < 2.0 ** -18
    assert np.array_equal(hz.data, seq.data) == (n == m)


def test_dense_plan_slot_algebra():
    # The plan's diagonals and pre-rotation reproduce W x in plain slot arithmetic.
    rng = np.random.default_rng(16)
    for m, n, n1, slots in [(4, 16, 2, 64), (64, 256, 8, 4096), (2, 64, 2, 4096), (8, 8, 8, 32)]:
        W = rng.normal(size=(m, n))
        x = rng.normal(size=n)
        xs = plan.input_slots(x, slots)
        pts = plan.plaintext_slots(W, n1, slots)
        z = np.zeros(slots)
        for j in range(m // n1):
            s = sum(pts[n1 * j + i] * np.roll(xs, -i) for i in range(n1))
            z = z + np.roll(s, -n1 * j)
        t = n // 2
        while t >= m:
            z = z + np.roll(z, -t)
            t //= 2
        assert np.allclose(z, plan.bias_slots(W @ x, slots))
    c = plan.op_counts(64, 256, 8)
    assert (c["baby"], c["giant"], c["rotate_and_sum"], c["multplain"]) == (7, 7, 2, 64)


def test_network_steps_cfg1():
    steps = ckks.network_steps(params.preset("cfg1").layers)
    assert steps == [1, 2, 3, 4, 5, 6, 7, 8, 16, 24, 32, 40, 48, 56, 64, 128]


# -------------------------------------------------------- the network
def test_network_cfg1_matches_fp64(oracle_lib):
    pr = params.preset("cfg1")
    o = ckks.Oracle(pr)
    rng = np.random.default_rng(2)
    Ws = [rng.normal(0, pr.sigma_w, (m, n)) for m, n, _ in pr.layers]
    bs = [rng.normal(0, pr.sigma_w, m) for m, _, _ in pr.layers]
    keys = o.keygen(1, ckks.network_steps(pr.layers))
    layers = o.prepare_network(Ws, bs, [l[2] for l in pr.layers])
    for r in range(2):
        x = np.random.default_rng(1000 + r).uniform(-1, 1, pr.layers[0][1])
        ct = o.encrypt(plan.input_slots(x, pr.slots), keys.pk, 5000 + r)
        out = o.eval_network(ct, layers, keys)
        assert out.level == 0
        y = o.decrypt_decode(out, keys.sk).real[:2]
        yr = plainnet.forward(x, Ws, bs)
        assert np.max(np.abs(y - yr)) <= 2.0 ** -12
        if abs(yr[0] - yr[1]) >= 2.0 ** -11:
            assert plainnet.predict(y) == plainnet.predict(yr)


# --------------------------------------------- cross-check with tiny.py
@pytest.mark.parametrize("log_n", [4, 5, 6])
def test_tiny_bit_exact(oracle_lib, log_n):
    pr = params.make(log_n, [50, 40, 40, 40], [50, 50], 2, 30)
    o = ckks.Oracle(pr)
    T = tiny.Tiny(pr.n, pr.q, pr.p, pr.alpha)
    m, n, n1 = 4, 8, 2
    steps = sorted(set(plan.rotation_steps(m, n, n1)) | {3})
    K = o.keygen(7, steps)
    s, pk, rlk, rot = T.keygen(7, steps)
    A = lambda v: np.array(v, dtype=np.uint64)
    assert K.sk.tolist() == s and np.array_equal(K.pk, A(pk)) and np.array_equal(K.rlk, A(rlk))
    for r in steps:
        assert np.array_equal(K.rot[r], A(rot[r]))
    rng = np.random.default_rng(log_n)
    x = rng.uniform(-1, 1, n)
    ct = o.encrypt(plan.input_slots(x, pr.slots), K.pk, 99)
    m_res = o.encode(plan.input_slots(x, pr.slots), pr.scale, pr.L)
    assert np.array_equal(ct.data, A(T.encrypt(m_res.tolist(), pk, 99)))
    L = pr.L
    c = ct.data.tolist()
    assert np.array_equal(o.decrypt(ct, K.sk), A(T.decrypt(c, s, L)))
    assert np.array_equal(o.rescale(ct).data, A(T.rescale(c, L)))
    for j in range(pr.dnum):
        assert np.array_equal(o.modup(ct.data[1], L, j), A(T.modup(c[1], L, j)))
    y = np.stack([rng.integers(0, q, pr.n, dtype=np.uint64) for q in pr.q + pr.p])
    assert np.array_equal(o.moddown(y, L), A(T.moddown(y.tolist(), L)))
    assert np.array_equal(o.keyswitch(ct.data[1], L, K.rlk), A(T.keyswitch(c[1], L, rlk)))
    assert np.array_equal(o.rotate(ct, 3, K).data, A(T.rotate(c, L, 3, rot)))
    assert np.array_equal(o.square(ct, K).data, A(T.square(c, L, rlk)))
    W = rng.normal(0, 0.1, (m, n))
    b = rng.normal(0, 0.1, m)
    lay = o.prepare_dense(W, b, n1, L, ct.scale)
    got = o.dense(ct, lay, K)
    want = T.dense(c, L, m, n, n1, lay.pts.tolist(), lay.bias.tolist(), rot)
    assert np.array_equal(got.data, A(want))
    # lazy-ModDown form: extended rotation and the dense layer
    assert np.array_equal(o.rotate_ext(ct, 3, K), A(T.rotate_ext(c, L, 3, rot)))
    assert np.array_equal(o.rotate_ext(ct, 0, K), A(T.rotate_ext(c, L, 0, rot)))
    lay_qp = o.prepare_dense(W, b, n1, L, ct.scale, qp=True)
    got = o.dense(ct, lay_qp, K)
    want = T.dense_qp(c, L, m, n, n1, lay_qp.pts.tolist(), lay_qp.bias.tolist(), rot)
    assert np.array_equal(got.data, A(want))
    # hoisted rotate-and-sum (2 -> period 2 from 8: shifts 2, 4, 6 in one group), both forms
    m3, n3, n13 = 2, 8, 2
    st3 = sorted(set(steps) | set(plan.rotation_steps(m3, n3, n13, 2)))
    K3 = o.keygen(7, st3)
    _, _, _, rot3 = T.keygen(7, st3)
    W3, b3 = rng.normal(0, 0.1, (m3, n3)), rng.normal(0, 0.1, m3)
    for qp in (False, True):
        lay3 = o.prepare_dense(W3, b3, n13, L, ct.scale, qp=qp, rs_bits=2)
        fn = T.dense_qp if qp else T.dense
        want = fn(c, L, m3, n3, n13, lay3.pts.tolist(), lay3.bias.tolist(), rot3, rs_bits=2)
        assert np.array_equal(o.dense(ct, lay3, K3).data, A(want)), qp
    # Two-layer network: dense -> rescale -> square -> rescale -> dense.
    W2 = rng.normal(0, 0.1, (2, m))
    b2 = rng.normal(0, 0.1, 2)
    layers = o.prepare_network([W, W2], [b, b2], [n1, 2])
    K2 = o.keygen(7, sorted(set(steps) | set(plan.rotation_steps(2, m, 2))))
    _, _, rlk2, rot2 = T.keygen(7, sorted(set(steps) | set(plan.rotation_steps(2, m, 2))))
    out = o.eval_network(ct, layers, K2)
    t = T.dense(c, L, m, n, n1, layers[0].pts.tolist(), layers[0].bias.tolist(), rot2)
    t = T.rescale(t, L)
    t = T.rescale(T.square(t, L - 1, rlk2), L - 1)
    t = T.rescale(T.dense(t, L - 2, 2, m, 2, layers[1].pts.tolist(), layers[1].bias.tolist(), rot2), L - 2)
    assert np.array_equal(out.data, A(t))

"""Pins of the oracle's client-side sampling (keys and encryption randomness).

The paper fixes none of it (Methods, "Experimental setting": 128-bit security
with SEAL); the reading used is SplitMix64 with one derived sub-seed per
sampled object, uniform residues by rejection, a uniform ternary secret and a
rounded Gaussian error of standard deviation 3.2 cut at |e| <= 19.  These
tests pin the oracle's C++ samplers against things other than their own
formulas:

  * the generator against the published SplitMix64 test vector;
  * each distribution by its statistics over 10^5 .. 10^6 draws (frequencies,
    moments, chi-square against the exact probability mass function), chosen
    so that a plausible mistake fails: a standard deviation of 32 or 0.32, a
    ternary draw that accepts the 2-bit value 3 (so 2 appears), a Gaussian
    cut at another bound, uniform residues without the rejection step (moduli
    near 2^64 make that bias large);
  * that keys and encryptions draw from these samplers: the public key's
    error b + a s, and an encryption's e0, e1 and v exposed by encrypting
    under a zero / unit public key.
"""
import ctypes as C
import math

import numpy as np
import pytest
from scipy import stats

from oracle import ckks, params

U64P = C.POINTER(C.c_uint64)
I64P = C.POINTER(C.c_int64)

# Chi-square p-values below this fail.  Every draw is seeded, so a test either
# passes or fails deterministically; the threshold only says how unlikely a
# correct sampler would have to be to fail.
P_FAIL = 1e-6


@pytest.fixture(scope="module")
def L(oracle_lib):
    lib = ckks.lib()
    lib.orc_sample_gaussian_sb.argtypes = [C.c_uint64, C.c_int, C.c_double, C.c_int64, I64P]
    lib.orc_noise_params.argtypes = [C.POINTER(C.c_double), I64P]
    lib.orc_sample_uniform_q.argtypes = [C.c_uint64, C.c_int, C.c_uint64, U64P]
    lib.orc_splitmix_stream.argtypes = [C.c_uint64, C.c_int, U64P]
    return lib


def _i64(n):
    a = np.empty(n, dtype=np.int64)
    return a, a.ctypes.data_as(I64P)


def ternary(L, seed, n):
    a, p = _i64(n)
    L.orc_sample_ternary(seed, n, p)
    return a


def gaussian(L, seed, n, sigma=None, bound=None):
    a, p = _i64(n)
    if sigma is None:
        L.orc_sample_gaussian(seed, n, p)
    else:
        L.orc_sample_gaussian_sb(seed, n, sigma, bound, p)
    return a


def uniform_q(L, seed, n, q):
    a = np.empty(n, dtype=np.uint64)
    L.orc_sample_uniform_q(seed, n, q, a.ctypes.data_as(U64P))
    return a


def rounded_normal_pmf(sigma, bound):
    """Exact pmf of round(N(0, sigma^2)) conditioned on |k| <= bound."""
    k = np.arange(-bound, bound + 1)
    cdf = stats.norm.cdf
    p = cdf((k + 0.5) / sigma) - cdf((k - 0.5) / sigma)
    return k, p / p.sum()


def chi2_pvalue(counts, probs, min_expected=20.0):
    """Chi-square goodness of fit; cells with small expectation are pooled."""
    n = counts.sum()
    exp = probs * n
    obs_c, exp_c, o_acc, e_acc = [], [], 0.0, 0.0
    for o, e in zip(counts, exp):
        o_acc += o
        e_acc += e
        if e_acc >= min_expected:
            obs_c.append(o_acc)
            exp_c.append(e_acc)
            o_acc = e_acc = 0.0
    if e_acc > 0:
        obs_c[-1] += o_acc
        exp_c[-1] += e_acc
    obs_c, exp_c = np.array(obs_c), np.array(exp_c)
    chi = float(((obs_c - exp_c) ** 2 / exp_c).sum())
    return float(stats.chi2.sf(chi, len(obs_c) - 1))


# ------------------------------------------------------------ generator
def test_splitmix64_published_vector(L):
    """The reference SplitMix64 (Steele, Lea and Flood; Vigna's public C
    version) seeded with 1234567 starts with these five outputs."""
    out = np.empty(5, dtype=np.uint64)
    L.orc_splitmix_stream(1234567, 5, out.ctypes.data_as(U64P))
    assert [int(v) for v in out] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                     4593380528125082431, 16408922859458223821]
    L.orc_splitmix_first.restype = C.c_uint64
    assert L.orc_splitmix_first(1234567) == 6457827717110365317


def test_sub_seeds_distinct_per_object(L):
    """Every sampled object of one key set, and of one encryption, gets its
    own stream: all sub-seeds under one master seed (tag level, then the
    per-polynomial level inside the C++ key and encryption routines) are
    distinct, for several master seeds, and streams of neighbouring tags are
    uncorrelated.  (Under the master-xor-tag rule two different masters can
    share a sub-seed, e.g. masters 1 and 2 with the rotation tags of steps 2
    and 1; a key set uses one master.)"""
    steps = [1, 2, 3, 7, 64, -1, -64, 255, 1 << 20]
    for master in (1, 2, 5000, 5001, 1 << 40):
        tags = [ckks.TAG_SECRET, ckks.TAG_PUBLIC, ckks.TAG_RELIN] + [ckks.tag_rotation(r) for r in steps]
        objs = [L.orc_derive_seed(master, t) for t in tags]
        assert len(set(objs)) == len(objs), "two objects share a sub-seed"
        allseeds = set(objs)
        for s in objs:
            # second level: public key (0x11, 0x12), switch keys per digit (0x100 + 2j, 0x101 + 2j)
            inner = [L.orc_derive_seed(s, u) for u in [0x11, 0x12] + [0x100 + i for i in range(16)]]
            assert len(set(inner)) == len(inner)
            allseeds |= set(inner)
        assert len(allseeds) == len(objs) * 19
        # encryption seed: v, e0, e1
        enc = [L.orc_derive_seed(master, u) for u in (0x21, 0x22, 0x23)]
        assert len(set(enc)) == 3
    # rotation tags keep the sign: +1 and -1 are different keys
    assert ckks.tag_rotation(1) != ckks.tag_rotation(-1)
    # streams of adjacent tags: correlation of the uniform outputs is ~0
    a = uniform_q(L, L.orc_derive_seed(7, 0x100), 200000, 1 << 62).astype(np.float64)
    b = uniform_q(L, L.orc_derive_seed(7, 0x101), 200000, 1 << 62).astype(np.float64)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.015


# -------------------------------------------------------------- ternary
def test_ternary_distribution(L):
    """Uniform on {-1, 0, 1}: support, each frequency within 1/3 +- 0.005 over
    10^6 draws (about 10 standard errors), chi-square, and no lag-1
    correlation.  Accepting the 2-bit value 3 would put 2 in the support and
    move every frequency to 1/4."""
    x = ternary(L, 0xA5A5, 1_000_000)
    vals, counts = np.unique(x, return_counts=True)
    assert list(vals) == [-1, 0, 1]
    freq = counts / x.size
    assert np.all(np.abs(freq - 1 / 3) < 0.005), freq
    assert chi2_pvalue(counts, np.full(3, 1 / 3)) > P_FAIL
    xf = x.astype(np.float64)
    assert abs(np.mean(xf[1:] * xf[:-1])) < 0.005


# ------------------------------------------------------------- gaussian
def test_noise_parameters():
    """The error distribution's declared constants (the reading: standard
    deviation 3.2, cut at 19 ~ 6 sigma), as the oracle library reports them."""
    lib = ckks.lib()
    lib.orc_noise_params.argtypes = [C.POINTER(C.c_double), I64P]
    s, b = C.c_double(), C.c_int64()
    lib.orc_noise_params(C.byref(s), C.byref(b))
    assert s.value == 3.2 and b.value == 19


def test_gaussian_default_distribution(L):
    """10^6 draws of the default error sampler: support within [-19, 19],
    mean 0, standard deviation sqrt(3.2^2 + 1/12) (rounding adds 1/12 to the
    variance), the mass beyond |e| >= 10, and a chi-square against the
    exact pmf of the rounded normal.  sigma = 32 or 0.32 fail every moment."""
    x = gaussian(L, 0x6A55, 1_000_000)
    assert np.max(np.abs(x)) <= 19
    assert abs(np.mean(x)) < 0.02
    want_std = math.sqrt(3.2 ** 2 + 1 / 12)
    assert abs(np.std(x) - want_std) < 0.02, np.std(x)
    tail = np.mean(np.abs(x) >= 10)
    want_tail = 2 * stats.norm.sf(9.5 / 3.2)
    assert abs(tail - want_tail) < 0.1 * want_tail, (tail, want_tail)
    k, p = rounded_normal_pmf(3.2, 19)
    counts = np.array([np.count_nonzero(x == v) for v in k])
    assert counts.sum() == x.size
    assert chi2_pvalue(counts, p) > P_FAIL


def test_gaussian_default_is_the_general_sampler(L):
    """The default sampler is the general one at the declared parameters:
    same stream bit for bit."""
    a = gaussian(L, 99, 100000)
    b = gaussian(L, 99, 100000, 3.2, 19)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("sigma,bound", [(8.0, 12), (3.2, 5), (20.0, 19)])
def test_gaussian_cut_is_rejection(L, sigma, bound):
    """Where the cut bites, draws beyond it are redrawn (not clamped, not
    folded): support within [-bound, bound], both ends reached, and the
    histogram equals the rounded normal conditioned on |k| <= bound."""
    x = gaussian(L, 1234 + bound, 400000, sigma, bound)
    assert np.max(np.abs(x)) == bound
    assert np.count_nonzero(x == bound) > 0 and np.count_nonzero(x == -bound) > 0
    k, p = rounded_normal_pmf(sigma, bound)
    counts = np.array([np.count_nonzero(x == v) for v in k])
    assert chi2_pvalue(counts, p) > P_FAIL
    # clamping would pile the cut mass onto +-bound: the end cells stay at their pmf
    end = (counts[0] + counts[-1]) / x.size
    assert abs(end - (p[0] + p[-1])) < 6 * math.sqrt((p[0] + p[-1]) / x.size) + 1e-4


# -------------------------------------------------------------- uniform
@pytest.mark.parametrize("q", [
    (1 << 50) - (1 << 17) + 1,          # a 50-bit NTT prime size (need not be prime here)
    0x6666666666666667,                 # ~0.4 * 2^64: without rejection [0, 0.2 * 2^64) gets 1.5x mass
    0xC000000000000001,                 # ~0.75 * 2^64: without rejection [0, 0.25 * 2^64) gets 2x mass
    3,
    1 << 63,                            # divides 2^64: every word accepted
])
def test_uniform_mod_distribution(L, q):
    """Residues below q, uniform over [0, q): chi-square over 64 equal buckets,
    mean (q - 1) / 2, and the low quarter's mass (where a missing or wrong
    rejection limit piles extra mass for moduli near 2^64)."""
    n = 400000
    x = uniform_q(L, 0x1111 + (q & 0xFFFF), n, q)
    assert int(x.max()) < q
    if q == 3:
        counts = np.bincount(x.astype(np.int64), minlength=3)
        assert chi2_pvalue(counts, np.full(3, 1 / 3)) > P_FAIL
        return
    buckets = np.minimum((x.astype(np.float64) / q * 64).astype(np.int64), 63)
    counts = np.bincount(buckets, minlength=64)
    assert chi2_pvalue(counts, np.full(64, 1 / 64)) > P_FAIL
    assert abs(np.mean(x.astype(np.float64)) / q - 0.5) < 0.005
    low = np.mean(x.astype(np.float64) < q / 4)
    assert abs(low - 0.25) < 0.005


def test_uniform_residues_of_keys(L):
    """The public key's a is uniform mod each prime (top bucket reached, chi-square)."""
    pr = params.make(13, [45, 35, 35, 35], [45], 1, 35)
    o = ckks.Oracle(pr)
    keys = o.keygen(3)
    a = keys.pk[1]
    for i, q in enumerate(pr.q):
        buckets = np.minimum((a[i].astype(np.float64) / q * 16).astype(np.int64), 15)
        assert chi2_pvalue(np.bincount(buckets, minlength=16), np.full(16, 1 / 16)) > P_FAIL
        assert int(a[i].max()) < q


# ------------------------------------------- samplers inside keys / encryption
def _centred(x, q):
    x = x.astype(np.int64) if q < (1 << 62) else x.astype(object)
    return np.where(x > q // 2, x - q, x)


def test_public_key_error_is_the_gaussian(L):
    """e = b + a s over q_0 (exact schoolbook negacyclic product, independent
    of the oracle's transform) is small, within the cut and of standard deviation ~3.2, and the
    secret is ternary with frequencies near 1/3."""
    pr = params.make(13, [45, 35, 35, 35], [45], 1, 35)
    o = ckks.Oracle(pr)
    keys = o.keygen(5)
    s = keys.sk
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == [-1, 0, 1] and np.all(np.abs(counts / s.size - 1 / 3) < 0.03)
    q = pr.q[0]
    b, a = keys.pk[0][0], keys.pk[1][0]
    # a s by schoolbook negacyclic convolution in int64: |a_i| < 2^45 and s is
    # ternary, so every partial sum stays below 2^58
    full = np.convolve(a.astype(np.int64), s.astype(np.int64))
    as_ = full[:pr.n].copy()
    as_[: pr.n - 1] -= full[pr.n:]
    e = _centred((b.astype(np.int64) + as_) % q, q)
    assert np.max(np.abs(e)) <= 19
    assert abs(np.std(e) - math.sqrt(3.2 ** 2 + 1 / 12)) < 0.1
    assert abs(np.mean(e)) < 0.15


def test_encryption_randomness_exposed(L):
    """Encrypting m = 0 under pk = (0, 0) gives (e0, e1); under pk = (1, 0)
    (the constant polynomial 1) gives (v + e0, e1): e0, e1 are two different
    draws of the error sampler and v is ternary."""
    pr = params.make(13, [45, 35, 35, 35], [45], 1, 35)
    o = ckks.Oracle(pr)
    N, nl = pr.n, len(pr.q)
    m = np.zeros((nl, N), dtype=np.uint64)

    def enc(pk, seed):
        ct = np.zeros((2, nl, N), dtype=np.uint64)
        L.orc_encrypt(o._h, pk.ctypes.data_as(U64P), m.ctypes.data_as(U64P), seed, ct.ctypes.data_as(U64P))
        return ct

    q0 = pr.q[0]
    pk0 = np.zeros((2, nl, N), dtype=np.uint64)
    ct = enc(pk0, 77)
    e0, e1 = _centred(ct[0][0], q0), _centred(ct[1][0], q0)
    for e in (e0, e1):
        assert np.max(np.abs(e)) <= 19 and abs(np.std(e) - math.sqrt(3.2 ** 2 + 1 / 12)) < 0.1
    assert not np.array_equal(e0, e1)
    assert abs(np.corrcoef(e0, e1)[0, 1]) < 0.05
    # the same integers on every limb (one small polynomial, reduced per prime)
    for i, q in enumerate(pr.q):
        assert np.array_equal(_centred(ct[0][i], q), e0)
    pk1 = pk0.copy()
    pk1[0, :, 0] = 1
    ct1 = enc(pk1, 77)
    v = _centred(ct1[0][0], q0) - e0
    vals, counts = np.unique(v, return_counts=True)
    assert list(vals) == [-1, 0, 1] and np.all(np.abs(counts / N - 1 / 3) < 0.03)
    assert np.array_equal(_centred(ct1[1][0], q0), e1)

"""Client path: encode, encrypt, decrypt and decode on the device.

CPU pins (no GPU): the oracle's encryption with given random polynomials
satisfies the exact decryption identity
    c0 + c1 s = m + v e_pk + e0 + e1 s   (mod q_i, as small integers),
with e_pk = b + a s recovered from the public key and every negacyclic
product formed by schoolbook integer convolution (numpy, exact in int64), so
a dropped term, a wrong sign or a swapped key half fails it.

GPU parity through the C ABI:
  * encode: integer coefficients within +-1 of the oracle's encoder (the
    device FFT and the oracle's FFT round differently; a coefficient whose
    scaled value lies within rounding of a half may go either way) and equal
    in all but a small fraction;
  * encrypt: bit for bit against the oracle given the same plaintext and the
    same random polynomials (exact modular arithmetic);
  * decrypt: bit for bit against the oracle's residues, at the top level and
    at lower levels;
  * decode: within 2^-30 of the oracle's FP64 decoder (both lift exactly;
    the FFTs differ by rounding, about log2(N) 2^-53 times the coefficient
    norm, far below the bound);
  * the whole client round trip around the small-net network replayed from
    its graph, against the FP64 plaintext network.
"""
import numpy as np
import pytest

from oracle import ckks, encode as enc, params, plan
from paper_2104_09164_amd import synth

MAX_ENC_DIFF_FRACTION = 1e-3


def negacyclic(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Schoolbook product in Z[X]/(X^N + 1) of int64 vectors (exact while the
    sums fit 63 bits)."""
    n = len(a)
    full = np.convolve(a.astype(np.int64), b.astype(np.int64))
    out = full[:n].copy()
    out[: n - 1] -= full[n:]
    return out


def centred(x: np.ndarray, q: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.int64) % q
    return np.where(x > q // 2, x - q, x)


def small_params():
    return params.make(10, [50] + [35] * 3, [50, 50], 2, 35)


@pytest.fixture(scope="module")
def o10(oracle_lib):
    return ckks.Oracle(small_params())


@pytest.fixture(scope="module")
def keys10(o10):
    return o10.keygen(11)


@pytest.mark.parametrize("level", [3, 1])
def test_encrypt_noise_decryption_identity(o10, keys10, level):
    pr = o10.pr
    n = pr.n
    qs = pr.q[: level + 1]
    s = keys10.sk.astype(np.int64)
    b, a = keys10.pk[0][0].astype(np.int64), keys10.pk[1][0].astype(np.int64)
    # a < 2^50 and s ternary: the schoolbook sums stay below 2^60
    e_pk = centred(b + negacyclic(a, s), pr.q[0])
    assert np.max(np.abs(e_pk)) <= 19
    v, e0, e1 = synth.encryption_noise(n, 31).astype(np.int64)
    assert set(np.unique(v)) <= {-1, 0, 1} and np.max(np.abs(e0)) <= 19
    m = synth.uniform_residues(qs, n, seed=32)
    ct = o10.encrypt_noise(m, keys10.pk, level, v, e0, e1, 2.0 ** 35)
    assert ct.data.shape == (2, level + 1, n) and ct.level == level
    noise = negacyclic(v, e_pk) + e0 + negacyclic(e1, s)
    dec = o10.decrypt(ct, keys10.sk)
    for i, q in enumerate(qs):
        want = (m[i].astype(object) + noise.astype(object)) % q
        assert np.array_equal(dec[i].astype(object), want), f"limb {i}"


def test_encrypt_noise_zero_noise_is_plaintext(o10, keys10):
    # v = e0 = e1 = 0: the ciphertext is (m, 0)
    n = o10.pr.n
    z = np.zeros(n, np.int64)
    m = synth.uniform_residues(o10.pr.q, n, seed=33)
    ct = o10.encrypt_noise(m, keys10.pk, o10.pr.L, z, z, z, 1.0)
    assert np.array_equal(ct.data[0], m) and not ct.data[1].any()


def test_noise_generator_ranges():
    nz = synth.encryption_noise(4096, 5)
    assert nz.dtype == np.int32 and nz.shape == (3, 4096)
    assert set(np.unique(nz[0])) == {-1, 0, 1}
    assert np.max(np.abs(nz[1:])) <= 19 and 2.5 < np.std(nz[1:]) < 4.0


# ------------------------------------------------------------------ GPU
def _ctx(pr):
    from paper_2104_09164_amd import he
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(4, 1, 1)
    return ctx


def _coeff_diff(got: np.ndarray, want: np.ndarray, qs) -> np.ndarray:
    """Signed integer difference of two residue arrays [l+1][N], checked to be
    one integer across all limbs and |d| <= 1."""
    d = None
    for i, q in enumerate(qs):
        di = centred(got[i].astype(np.int64) - want[i].astype(np.int64), q)
        if d is None:
            d = di
        assert np.array_equal(di, d), f"limb {i} disagrees on the integer difference"
    assert np.max(np.abs(d)) <= 1
    return d


ENC_CASES = [
    # (log_n, q bits, p bits, alpha, scale bits, level, requests)
    (10, [50, 35, 35, 35], [50, 50], 2, 35, 3, 3),
    (12, [50, 40, 40, 40], [50, 50], 2, 40, 2, 2),
    (15, [60] + [40] * 6, [60, 60], 2, 40, 6, 2),      # the small net's ring
    (16, [50] * 24, [50] * 8, 8, 40, 23, 1),           # the key-switch ring: 24 limbs (memory-resident digits)
]


@pytest.mark.gpu
@pytest.mark.parametrize("case", ENC_CASES, ids=[f"n{c[0]}_l{c[5]}" for c in ENC_CASES])
def test_encode_within_one(case):
    import torch
    log_n, qb, pb, alpha, sb, level, R = case
    pr = params.make(log_n, qb, pb, alpha, sb)
    print(f"[client] encode N=2^{log_n} level {level} x{R}", flush=True)
    ctx = _ctx(pr)
    cl = ctx.client(R)
    zs = synth.slot_vectors(R, pr.slots, 40 + log_n)
    scale = 2.0 ** sb
    pt = cl.encode(torch.from_numpy(zs), scale, level).cpu().numpy().view(np.uint64)
    qs = pr.q[: level + 1]
    mism = 0
    for r in range(R):
        want = enc.encode(zs[r], scale, qs, pr.n)
        d = _coeff_diff(pt[r], want, qs)
        mism += int(np.count_nonzero(d))
    assert mism <= MAX_ENC_DIFF_FRACTION * R * pr.n


@pytest.mark.gpu
@pytest.mark.parametrize("case", ENC_CASES[:3], ids=[f"n{c[0]}_l{c[5]}" for c in ENC_CASES[:3]])
def test_encrypt_bit_exact(case):
    import torch
    log_n, qb, pb, alpha, sb, level, R = case
    pr = params.make(log_n, qb, pb, alpha, sb)
    o = ckks.Oracle(pr)
    keys = o.keygen(7, relin=False)
    print(f"[client] encrypt N=2^{log_n} level {level} x{R}", flush=True)
    ctx = _ctx(pr)
    cl = ctx.client(R, pk=keys.pk)
    scale = 2.0 ** sb
    zs = synth.slot_vectors(R, pr.slots, 50)
    for lev in sorted({level, max(0, level - 1)}):
        qs = pr.q[: lev + 1]
        ms = np.stack([o.encode(zs[r], scale, lev) for r in range(R)])
        noise = np.stack([synth.encryption_noise(pr.n, 60 + r) for r in range(R)])
        outs = cl.encrypt(torch.from_numpy(ms.view(np.int64)).cuda(), torch.from_numpy(noise).cuda(), lev, scale)
        for r in range(R):
            want = o.encrypt_noise(ms[r], keys.pk, lev, *noise[r], scale)
            got = ctx.export_ct(outs[r])
            assert outs[r].level == lev and outs[r].scale == scale
            assert np.array_equal(got, want.data), f"request {r} level {lev} differs from the oracle"
            assert len(qs) == got.shape[1]


@pytest.mark.gpu
@pytest.mark.parametrize("case", ENC_CASES[:3], ids=[f"n{c[0]}_l{c[5]}" for c in ENC_CASES[:3]])
def test_decrypt_bit_exact_and_decode(case):
    import torch
    log_n, qb, pb, alpha, sb, level, R = case
    pr = params.make(log_n, qb, pb, alpha, sb)
    o = ckks.Oracle(pr)
    keys = o.keygen(8, relin=False)
    print(f"[client] decrypt N=2^{log_n} level {level} x{R}", flush=True)
    ctx = _ctx(pr)
    cl = ctx.client(R, sk=keys.sk)
    zs = synth.slot_vectors(R, pr.slots, 70)
    top = [o.encrypt(zs[r], keys.pk, 90 + r) for r in range(R)]
    for lev in sorted({level, level - 1, 0}, reverse=True):
        # the top-level ciphertext restricted to q_0..q_lev encrypts the same
        # message at the same scale
        cts = [ckks.Ciphertext(np.ascontiguousarray(c.data[:, : lev + 1]), lev, c.scale) for c in top]
        scale = cts[0].scale
        dev = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
        pt = cl.decrypt(dev)
        got = pt.cpu().numpy().view(np.uint64)
        z = cl.decode(pt, lev, scale).cpu().numpy()
        for r in range(R):
            want = o.decrypt(cts[r], keys.sk)
            assert np.array_equal(got[r], want), f"request {r} level {lev}: residues differ"
            zw = enc.decode(want, scale, pr.q[: lev + 1], pr.n)
            assert np.max(np.abs(z[r] - zw)) <= 2.0 ** -30
            assert np.max(np.abs(z[r] - zs[r])) < 2.0 ** -10


@pytest.mark.gpu
def test_decode_large_values_and_signs():
    """Exact centred lift of positive and negative coefficients up to about
    2^57 over 24 limbs (Q ~ 2^1200, digits kept in per-lane memory), two limbs
    and one limb: decode of oracle encodings against the oracle's decoder."""
    import torch
    pr = params.make(16, [50] * 24, [50] * 8, 8, 40)
    ctx = _ctx(pr)
    cl = ctx.client(1)
    z = synth.slot_vectors(1, pr.slots, 80)[0] * 4.0
    for lev, sb in ((23, 60), (1, 55), (0, 45)):
        qs = pr.q[: lev + 1]
        want_pt = enc.encode(z, 2.0 ** sb, qs, pr.n)
        pt = torch.from_numpy(want_pt[None].view(np.int64)).cuda()
        got = cl.decode(pt, lev, 2.0 ** sb).cpu().numpy()[0]
        want = enc.decode(want_pt, 2.0 ** sb, qs, pr.n)
        rel = np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert rel <= 2.0 ** -40, f"level {lev}: relative error {rel}"


@pytest.mark.gpu
def test_client_max_batch():
    """The largest batch (64 requests per call) at N = 2^10: encryption bit
    for bit, decryption bit for bit, decode within the bound, for every
    request."""
    import torch
    from paper_2104_09164_amd import he
    pr = small_params()
    o = ckks.Oracle(pr)
    keys = o.keygen(12, relin=False)
    ctx = _ctx(pr)
    R = he.HE_MAX_BATCH
    cl = ctx.client(R, pk=keys.pk, sk=keys.sk)
    print(f"[client] max batch {R}", flush=True)
    zs = synth.slot_vectors(R, pr.slots, 90)
    ms = np.stack([o.encode(zs[r], pr.scale, pr.L) for r in range(R)])
    noise = np.stack([synth.encryption_noise(pr.n, 200 + r) for r in range(R)])
    outs = cl.encrypt(torch.from_numpy(ms.view(np.int64)).cuda(), torch.from_numpy(noise).cuda(), pr.L, pr.scale)
    pt = cl.decrypt(outs)
    z = cl.decode(pt, pr.L, pr.scale).cpu().numpy()
    got_pt = pt.cpu().numpy().view(np.uint64)
    for r in range(R):
        ct = o.encrypt_noise(ms[r], keys.pk, pr.L, *noise[r], pr.scale)
        assert np.array_equal(ctx.export_ct(outs[r]), ct.data), f"request {r}: ciphertext"
        want = o.decrypt(ct, keys.sk)
        assert np.array_equal(got_pt[r], want), f"request {r}: residues"
        assert np.max(np.abs(z[r] - enc.decode(want, pr.scale, pr.q, pr.n))) <= 2.0 ** -30


@pytest.mark.gpu
def test_client_errors():
    import torch
    from paper_2104_09164_amd import he
    pr = small_params()
    ctx = _ctx(pr)
    o = ckks.Oracle(pr)
    keys = o.keygen(9, relin=False)
    cl = ctx.client(2)                       # no keys
    pt = torch.zeros((1, pr.L + 1, pr.n), dtype=torch.int64, device="cuda")
    nz = torch.zeros((1, 3, pr.n), dtype=torch.int32, device="cuda")
    with pytest.raises(he.HeError) as e:
        cl.encrypt(pt, nz, pr.L, 1.0)
    assert e.value.code == -3
    with pytest.raises(he.HeError) as e:
        cl.decrypt([ctx.new_ct(pr.L)])
    assert e.value.code == -3
    with pytest.raises(he.HeError) as e:     # level beyond L
        cl.encode(torch.zeros((1, pr.slots), dtype=torch.complex128), 2.0 ** 30, pr.L + 1)
    assert e.value.code == -4
    with pytest.raises(he.HeError) as e:     # batch beyond max_batch
        cl.encode(torch.zeros((3, pr.slots), dtype=torch.complex128), 2.0 ** 30, 0)
    assert e.value.code == -1
    with pytest.raises(he.HeError) as e:
        ctx.client(2, sk=np.full(pr.n, 2, dtype=np.int64))
    assert e.value.code == -1
    bad_pk = keys.pk.copy()
    bad_pk[1, 2, 5] = pr.q[2]                # a residue equal to its prime
    with pytest.raises(he.HeError) as e:
        ctx.client(2, pk=bad_pk)
    assert e.value.code == -1
    # misaligned slot arrays are rejected before anything is enqueued
    zbuf = torch.zeros(pr.slots + 1, dtype=torch.complex128, device="cuda")
    out = torch.zeros((1, 1, pr.n), dtype=torch.int64, device="cuda")
    import ctypes
    rc = he.lib().he_encode(cl.h, 1, ctypes.c_void_p(zbuf.data_ptr() + 8), 2.0 ** 30, 0,
                            ctypes.c_void_p(out.data_ptr()))
    assert rc == -1
    rc = he.lib().he_decode(cl.h, 1, ctypes.c_void_p(out.data_ptr()), 0, 2.0 ** 30,
                            ctypes.c_void_p(zbuf.data_ptr() + 8))
    assert rc == -1
    with pytest.raises(he.HeError) as e:     # scale must be positive and finite
        cl.encode(torch.zeros((1, pr.slots), dtype=torch.complex128), 0.0, 0)
    assert e.value.code == -1
    # empty batches are no-ops
    cl2 = ctx.client(2, pk=keys.pk, sk=keys.sk)
    assert cl2.encode(torch.zeros((0, pr.slots), dtype=torch.complex128), 2.0 ** 30, 0).shape[0] == 0
    assert cl2.decrypt([]).shape[0] == 0


@pytest.mark.gpu
def test_client_round_trip_small_net():
    """End users encode and encrypt on the device, the network runs from its
    graph, the monitoring service decrypts and decodes on the device: logits
    within 2^-12 of the FP64 network, and bit-identical network outputs to
    the oracle's encryption path when given the oracle's plaintexts."""
    import torch
    from paper_2104_09164_amd import he, netplan, tune
    from paper_2104_09164_amd.batch import NetworkRunner
    from oracle import plainnet
    name = "cfg3"
    c = netplan.PRESETS[name]
    tuned = tune.load(name, "gfx950")
    shapes = netplan.tuned_shapes(name, tuned, False)
    pr = params.preset(name)
    o = ckks.Oracle(pr)
    rs = [s[4] if len(s) > 4 else 0 for s in shapes]
    steps = ckks.network_steps([s[:3] for s in shapes], rs)
    print(f"[client] round trip {name}: keygen", flush=True)
    keys = o.keygen(synth.SEED_KEYS, steps)
    Ws, bs = synth.network_weights([s[:3] for s in shapes], c["sigma"])
    lays = o.prepare_network(Ws, bs, [s[2] for s in shapes], qps=[len(s) > 3 and s[3] for s in shapes], rs_bits=rs)
    npl = netplan.plan_network(pr.log_n, pr.q, pr.p, pr.alpha, c["scale_bits"], shapes)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    tune.apply_knobs(ctx, tuned)
    B = 4
    ctx.bind(B, npl.max_n1(), npl.max_n2())
    ctx.load_keys(keys.rlk, keys.rot)
    dls = [ctx.dense_load(l.level, l.m, l.n, l.n1, l.pts, l.bias, l.pt_scale, l.bias_scale, qp=l.qp, rs_bits=l.rs_bits)
           for l in lays]
    runner = NetworkRunner(ctx, npl, dls, B)
    cl = ctx.client(B, pk=keys.pk, sk=keys.sk)
    xs = [synth.request_input(shapes[0][1], r) for r in range(B)]
    z = torch.from_numpy(np.stack([plan.input_slots(x, pr.slots) for x in xs]).astype(np.complex128))
    noise = torch.from_numpy(np.stack([synth.encryption_noise(pr.n, 100 + r) for r in range(B)])).cuda()
    pt = cl.encode(z, pr.scale, pr.L)
    cl.encrypt(pt, noise, pr.L, pr.scale, outs=runner.inputs[:B])
    g = runner.capture(B)
    g.replay()
    torch.cuda.synchronize()
    outs = runner.outputs(B)
    y = cl.decode(cl.decrypt(outs), npl.out_level, npl.out_scale).cpu().numpy()
    for r in range(B):
        yr = plainnet.forward(xs[r], Ws, bs)
        assert np.max(np.abs(y[r].real[:2] - yr)) <= 2.0 ** -12
    # the same network on the oracle's plaintext of request 0: bit for bit
    m0 = o.encode(plan.input_slots(xs[0], pr.slots), pr.scale, pr.L)
    nz0 = synth.encryption_noise(pr.n, 100)
    ct0 = o.encrypt_noise(m0, keys.pk, pr.L, *nz0, pr.scale)
    cl.encrypt(torch.from_numpy(m0[None].view(np.int64)).cuda(), torch.from_numpy(nz0[None]).cuda(), pr.L,
               pr.scale, outs=runner.inputs[:1])
    g.replay()
    torch.cuda.synchronize()
    print(f"[client] round trip {name}: oracle network", flush=True)
    want = o.eval_network(ct0, lays, keys)
    assert np.array_equal(ctx.export_ct(runner.outputs(B)[0]), want.data)

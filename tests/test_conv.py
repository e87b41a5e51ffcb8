"""Multi-channel homomorphic convolution (the paper's convolution equation in
its baby-step strategy) through the multi-input linear transform.

CPU: the layout and pre-rotation algebra on plain slot vectors against a
direct FP64 1-D convolution; the oracle's RNS-CKKS evaluation decrypts to it.
GPU: he_eval_linear bit for bit against the oracle (small ring, several
inputs and outputs), and at the 1D-CNN-64 layer shapes of the paper's
Table 1 (N = 2^15) on sampled outputs.
"""
import numpy as np
import pytest

from oracle import ckks, conv, params

SMALL = dict(c=4, dist=16, L=12, f=3, n_in=2, n_out=2)


def _case(pr, c, dist, L, f, n_in, n_out, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (c * n_in, L))
    W = rng.normal(0, 0.1, (c * n_out, c * n_in, f))
    baby, giant = conv.rotations(f, c, dist)
    return X, W, baby, giant


@pytest.mark.parametrize("c,dist,L,f,n_in,n_out", [(4, 16, 12, 3, 2, 2), (2, 8, 5, 5, 3, 1), (8, 32, 30, 3, 1, 2)])
def test_conv_slot_model_equals_fp64(c, dist, L, f, n_in, n_out):
    slots = 512
    X, W, baby, giant = _case(None, c, dist, L, f, n_in, n_out, 1)
    xs = conv.pack(X, c, dist, slots)
    pts = conv.plaintext_slots(W, c, dist, L, slots)
    outs = conv.slot_model(xs, pts, baby, giant)
    want = conv.conv1d_fp64(X, W)
    for j, v in enumerate(outs):
        assert np.allclose(conv.unpack(v, c, dist, L), want[j * c:(j + 1) * c], atol=1e-12)
        # the block is replicated across the slots, padding stays zero
        blk = v[:c * dist]
        assert np.allclose(v, np.tile(blk, slots // (c * dist)), atol=1e-12)
        assert np.allclose(blk.reshape(c, dist)[:, L:], 0)


def _small_params():
    return params.make(10, [50, 40, 40, 40, 40], [50, 50, 50], 3, 35)


def test_conv_oracle_decrypts(oracle_lib):
    pr = _small_params()
    o = ckks.Oracle(pr)
    X, W, baby, giant = _case(pr, seed=2, **SMALL)
    c, dist, L = SMALL["c"], SMALL["dist"], SMALL["L"]
    keys = o.keygen(3, sorted(set(baby + giant) - {0}))
    cts = [o.encrypt(v, keys.pk, 40 + i) for i, v in enumerate(conv.pack(X, c, dist, pr.slots))]
    pts = conv.encode_plaintexts(o, conv.plaintext_slots(W, c, dist, L, pr.slots), pr.scale, pr.L)
    outs = o.linear(cts, pts, baby, giant, pr.scale, keys)
    want = conv.conv1d_fp64(X, W)
    for j, ct in enumerate(outs):
        got = o.decrypt_decode(o.rescale(ct), keys.sk).real
        assert np.max(np.abs(conv.unpack(got, c, dist, L) - want[j * c:(j + 1) * c])) < 2.0 ** -14


@pytest.mark.gpu
def test_conv_gpu_parity_small():
    from paper_2104_09164_amd import he
    pr = _small_params()
    o = ckks.Oracle(pr)
    X, W, baby, giant = _case(pr, seed=4, **SMALL)
    c, dist, L, n_in, n_out = SMALL["c"], SMALL["dist"], SMALL["L"], SMALL["n_in"], SMALL["n_out"]
    keys = o.keygen(3, sorted(set(baby + giant) - {0}))
    cts = [o.encrypt(v, keys.pk, 60 + i) for i, v in enumerate(conv.pack(X, c, dist, pr.slots))]
    pts = conv.encode_plaintexts(o, conv.plaintext_slots(W, c, dist, L, pr.slots), pr.scale, pr.L)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(max(n_in, n_out), 1, len(giant))
    ctx.load_keys(None, keys.rot)
    lt = ctx.linear_load(pr.L, baby, giant, pts, pr.scale)
    gs = [ctx.import_ct(ct.data, ct.level, ct.scale) for ct in cts]
    outs = ctx.eval_linear(gs, lt)
    want = o.linear(cts, pts, baby, giant, pr.scale, keys)
    for j in range(n_out):
        assert outs[j].scale == want[j].scale and outs[j].level == want[j].level
        assert np.array_equal(ctx.export_ct(outs[j]), want[j].data), j
    # a second call (rotation scratch reused) gives the same words
    again = ctx.eval_linear(gs, lt)
    assert np.array_equal(ctx.export_ct(again[1]), want[1].data)
    # two requests batched over the same plaintexts: each equals its single evaluation
    cts2 = [o.encrypt(v, keys.pk, 70 + i) for i, v in enumerate(conv.pack(X[::-1].copy(), c, dist, pr.slots))]
    gs2 = [ctx.import_ct(ct.data, ct.level, ct.scale) for ct in cts2]
    ctx.bind(2 * max(n_in, n_out), 1, len(giant))
    both = ctx.eval_linear_batch(gs + gs2, lt)
    single2 = ctx.eval_linear(gs2, lt)
    for j in range(n_out):
        assert np.array_equal(ctx.export_ct(both[j]), want[j].data)
        assert np.array_equal(ctx.export_ct(both[n_out + j]), ctx.export_ct(single2[j]))
    assert np.array_equal(ctx.export_ct(both[n_out]), o.linear(cts2, pts, baby, giant, pr.scale, keys, only=[0])[0].data)


@pytest.mark.gpu
@pytest.mark.parametrize("layer", ["1d64_conv2", "1d64_conv3"])
def test_conv_gpu_table1_shapes(layer):
    """1D-CNN-64 conv2 (map 240, 64 -> 128 channels, n_in 4, n_out 8) and
    conv3 (map 120, 128 -> 256, n_in 8, n_out 16), 16 channels per
    ciphertext, kernel width 3, N = 2^15 (the small net's ring): the first
    and last output ciphertexts bit for bit against the oracle and within
    2^-12 of the FP64 convolution."""
    from paper_2104_09164_amd import he, netplan
    L, n_in, n_out = {"1d64_conv2": (240, 4, 8), "1d64_conv3": (120, 8, 16)}[layer]
    c, f = 16, 3
    dist = 1 << (L - 1).bit_length()
    pr = params.preset("cfg3")
    o = ckks.Oracle(pr)
    X, W, baby, giant = _case(pr, c, dist, L, f, n_in, n_out, 7)
    print(f"[conv] {layer}: keygen", flush=True)
    keys = o.keygen(3, sorted(set(baby + giant) - {0}), relin=False)
    cts = [o.encrypt(v, keys.pk, 80 + i) for i, v in enumerate(conv.pack(X, c, dist, pr.slots))]
    print(f"[conv] {layer}: encoding {c * n_out * n_in * f} plaintexts", flush=True)
    pts = conv.encode_plaintexts(o, conv.plaintext_slots(W, c, dist, L, pr.slots), pr.scale, pr.L)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(max(n_in, n_out), 1, c)
    ctx.load_keys(None, keys.rot)
    lt = ctx.linear_load(pr.L, baby, giant, pts, pr.scale)
    outs = ctx.eval_linear([ctx.import_ct(ct.data, ct.level, ct.scale) for ct in cts], lt)
    print(f"[conv] {layer}: oracle outputs 0 and {n_out - 1}", flush=True)
    want = o.linear(cts, pts, baby, giant, pr.scale, keys, only=[0, n_out - 1])
    ref = conv.conv1d_fp64(X, W)
    for w, j in zip(want, [0, n_out - 1]):
        got = ctx.export_ct(outs[j])
        assert np.array_equal(got, w.data), j
        dec = o.decrypt_decode(o.rescale(ckks.Ciphertext(got, outs[j].level, outs[j].scale)), keys.sk).real
        assert np.max(np.abs(conv.unpack(dec, c, dist, L) - ref[j * c:(j + 1) * c])) < 2.0 ** -12


# ------------------------------------------------------------- fast convolution
FAST_SMALL = dict(c=4, dist=32, Lp=6, f=3, n_in=4, n_out=2, nP=2)


def _fast_case(c, dist, Lp, f, n_in, n_out, nP, seed, slots):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (c * n_in, Lp))
    W = rng.normal(0, 0.1, (c * n_out, c * n_in, f))
    xs = conv.pack_punctured(X, c, dist, nP, slots, rng)
    return X, W, xs


@pytest.mark.parametrize("c,dist,Lp,f,n_in,n_out,nP", [(4, 32, 6, 3, 4, 2, 4), (2, 16, 5, 3, 2, 1, 2),
                                                        (4, 64, 10, 5, 4, 2, 2)])
def test_fast_conv_slot_model_equals_fp64(c, dist, Lp, f, n_in, n_out, nP):
    # merge (mask, shift, sum), convolve the merged ciphertexts, rotate-and-sum:
    # on plain slot vectors with junk at the punctured positions, the valid
    # positions equal the FP64 convolution of the pooled maps
    slots = 512
    X, W, xs = _fast_case(c, dist, Lp, f, n_in, n_out, nP, 3, slots)
    rot = conv.fast_rotations(f, c, dist, nP)
    mp, _ = conv.merge_plaintext_slots(c, dist, Lp, nP, slots)
    merged = [conv.slot_model(xs[a * nP:(a + 1) * nP], mp, [0], rot["pre"])[0] for a in range(n_in // nP)]
    outs = conv.slot_model(merged, conv.fast_plaintext_slots(W, c, dist, Lp, nP, slots), rot["baby"], rot["giant"])
    want = conv.conv1d_fp64(X, W)
    for j, z in enumerate(outs):
        for t in rot["post"]:
            z = z + np.roll(z, -t)
        assert np.allclose(conv.unpack_punctured(z, c, dist, Lp, nP), want[j * c:(j + 1) * c], atol=1e-12)


def _fast_params():
    # scale = the 40-bit primes, so the two rescales of the fast convolution keep it at 2^40
    return params.make(10, [50, 40, 40, 40, 40], [50, 50, 50], 3, 40)


def _fast_setup(o, pr, case, seed):
    X, W, xs = _fast_case(**case, seed=seed, slots=pr.slots)
    c, dist, Lp, f, nP = case["c"], case["dist"], case["Lp"], case["f"], case["nP"]
    rot = conv.fast_rotations(f, c, dist, nP)
    mp, _ = conv.merge_plaintext_slots(c, dist, Lp, nP, pr.slots)
    pre = conv.encode_plaintexts(o, mp, pr.scale, pr.L)
    fast = conv.encode_plaintexts(o, conv.fast_plaintext_slots(W, c, dist, Lp, nP, pr.slots), pr.scale, pr.L - 1)
    return X, W, xs, rot, pre, fast


def test_fast_conv_oracle_decrypts(oracle_lib):
    pr = _fast_params()
    o = ckks.Oracle(pr)
    X, W, xs, rot, pre, fast = _fast_setup(o, pr, FAST_SMALL, 5)
    keys = o.keygen(3, sorted(set(rot["pre"] + rot["baby"] + rot["giant"] + rot["post"]) - {0}))
    cts = [o.encrypt(v, keys.pk, 90 + i) for i, v in enumerate(xs)]
    _, outs = conv.fast_conv(o, cts, pre, fast, rot, pr.scale, keys)
    want = conv.conv1d_fp64(X, W)
    c, dist, Lp, nP = FAST_SMALL["c"], FAST_SMALL["dist"], FAST_SMALL["Lp"], FAST_SMALL["nP"]
    for j, ct in enumerate(outs):
        got = o.decrypt_decode(ct, keys.sk).real
        assert np.max(np.abs(conv.unpack_punctured(got, c, dist, Lp, nP) - want[j * c:(j + 1) * c])) < 2.0 ** -14


def _gpu_fast(ctx, pr, case, rot, pre, fast, gcts):
    from paper_2104_09164_amd.conv import FastConv
    fc = FastConv(ctx, pr.L, case["nP"], rot["pre"], pre, rot["baby"], rot["giant"], fast, rot["post"], pr.scale)
    return fc, fc.run(gcts)


@pytest.mark.gpu
def test_fast_conv_gpu_parity_small():
    from paper_2104_09164_amd import he
    pr = _fast_params()
    o = ckks.Oracle(pr)
    X, W, xs, rot, pre, fast = _fast_setup(o, pr, FAST_SMALL, 6)
    keys = o.keygen(3, sorted(set(rot["pre"] + rot["baby"] + rot["giant"] + rot["post"]) - {0}))
    cts = [o.encrypt(v, keys.pk, 95 + i) for i, v in enumerate(xs)]
    merged_w, outs_w = conv.fast_conv(o, cts, pre, fast, rot, pr.scale, keys)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    n_in, n_out, nP = FAST_SMALL["n_in"], FAST_SMALL["n_out"], FAST_SMALL["nP"]
    ctx.bind(max(n_in, n_out), 1, max(nP, FAST_SMALL["c"]))      # the merge step batches all n_in inputs
    ctx.load_keys(None, keys.rot)
    fc, outs = _gpu_fast(ctx, pr, FAST_SMALL, rot, pre, fast, [ctx.import_ct(c.data, c.level, c.scale) for c in cts])
    for a, m in enumerate(merged_w):
        assert np.array_equal(ctx.export_ct(fc.merged[a]), m.data), a
    for j, w in enumerate(outs_w):
        assert outs[j].level == w.level and outs[j].scale == w.scale
        assert np.array_equal(ctx.export_ct(outs[j]), w.data), j


@pytest.mark.gpu
def test_fast_conv_gpu_table1_1d64_conv3():
    """1D-CNN-64 conv3 with the fast convolution (Table 1: n_in 8, n_out 16,
    load number n_P = 4): pooled maps of 120 at stride 4 (slot distance 512),
    16 channels per ciphertext, kernel width 3, N = 2^15: merged ciphertexts
    and the first and last outputs bit for bit against the oracle, and within
    2^-12 of the FP64 convolution."""
    from paper_2104_09164_amd import he
    pr = params.preset("cfg3")
    o = ckks.Oracle(pr)
    case = dict(c=16, dist=512, Lp=120, f=3, n_in=8, n_out=16, nP=4)
    print("[conv] fast conv3: plaintexts", flush=True)
    X, W, xs, rot, pre, fast = _fast_setup(o, pr, case, 8)
    keys = o.keygen(3, sorted(set(rot["pre"] + rot["baby"] + rot["giant"] + rot["post"]) - {0}), relin=False)
    cts = [o.encrypt(v, keys.pk, 120 + i) for i, v in enumerate(xs)]
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(32, 1, 16)
    ctx.load_keys(None, keys.rot)
    gcts = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
    fc, outs = _gpu_fast(ctx, pr, case, rot, pre, fast, gcts + gcts[::-1])     # two requests in one batch
    assert len(outs) == 32
    print("[conv] fast conv3: oracle", flush=True)
    merged_w, outs_w = conv.fast_conv(o, cts, pre, fast, rot, pr.scale, keys, only=[0, 15])
    for a, m in enumerate(merged_w):
        assert np.array_equal(ctx.export_ct(fc.merged[a]), m.data), a
    want = conv.conv1d_fp64(X, W)
    for w, j in zip(outs_w, [0, 15]):
        got = ctx.export_ct(outs[j])
        assert np.array_equal(got, w.data), j
        dec = o.decrypt_decode(ckks.Ciphertext(got, outs[j].level, outs[j].scale), keys.sk).real
        assert np.max(np.abs(conv.unpack_punctured(dec, 16, 512, 120, 4) - want[j * 16:(j + 1) * 16])) < 2.0 ** -12

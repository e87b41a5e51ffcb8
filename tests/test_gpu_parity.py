"""GPU parity: every C-ABI operation against the CPU oracle, bit for bit.

Inputs (keys, ciphertexts, encoded plaintexts) come from the oracle's client
side and seeded generators; the GPU path receives them through the C ABI in
coefficient form and its outputs are exported in coefficient form, so equality
is element-by-element on the unique representation.
"""
import numpy as np
import pytest

from oracle import ckks, params, plainnet, plan
from paper_2104_09164_amd import synth

pytestmark = pytest.mark.gpu


def _he():
    from paper_2104_09164_amd import he
    return he


def make_setup(pr, steps, max_batch=4, max_n1=8, max_n2=8, relin=True, seed=1):
    he = _he()
    o = ckks.Oracle(pr)
    keys = o.keygen(seed, steps, relin=relin)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(max_batch, max_n1, max_n2)
    ctx.load_keys(keys.rlk, keys.rot)
    return o, keys, ctx


# nq = 5, K = 3, alpha = 3: digits {0,1,2}, {3,4}; at level 3 the last digit is {3} (ragged).
def small(log_n=10):
    return params.make(log_n, [50, 40, 40, 40, 40], [50, 50, 50], 3, 35)


DENSE_CASES = [(8, 64, 4, True), (8, 64, 1, True), (8, 64, 8, False), (16, 16, 4, True), (2, 8, 2, True),
               (2, 8, 1, False)]


@pytest.fixture(scope="module")
def setup10():
    pr = small(10)
    steps = {1, 2, 3, 5, 7, 64, 100, -1, 255}
    for m, n, n1, _ in DENSE_CASES:
        steps |= set(plan.rotation_steps(m, n, n1))
    return (pr,) + make_setup(pr, sorted(steps))


def encrypt(o, keys, pr, seed, width=None):
    x = synth.request_input(width or pr.slots, seed)
    return x, o.encrypt(plan.input_slots(x, pr.slots), keys.pk, synth.request_seed(seed))


@pytest.mark.parametrize("log_n", [10, 11, 12, 13, 14, 15, 16])
def test_ntt_roundtrip_and_convolution(log_n):
    import torch
    he = _he()
    pr = params.make(log_n, [60, 45], [61], 1, 30)
    o = ckks.Oracle(pr)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    rng = np.random.default_rng(log_n)
    primes = pr.q + pr.p
    a = synth.uniform_residues(primes, pr.n, (), seed=log_n)
    b = synth.uniform_residues(primes, pr.n, (), seed=100 + log_n)
    ab = o.polymul(a, b, list(range(len(primes))))
    bufs = [torch.from_numpy(x.view(np.int64).copy()).to("cuda") for x in (a, b, ab)]
    ctx.ntt(bufs, 0, len(primes), inverse=False)
    ctx.sync()
    A, B, AB = [x.cpu().numpy().view(np.uint64).reshape(len(primes), pr.n) for x in bufs]
    for i, q in enumerate(primes):
        assert A[i].max() < q
        prod = (A[i].astype(object) * B[i].astype(object)) % q
        assert np.array_equal(prod.astype(np.uint64), AB[i]), f"NTT is not a ring map at prime {i}"
    ctx.ntt(bufs[:1], 0, len(primes), inverse=True)
    ctx.sync()
    assert np.array_equal(bufs[0].cpu().numpy().view(np.uint64).reshape(len(primes), pr.n), a)
    if log_n == 15:
        # the register-resident single-pass transform gives the same words as the two-phase one
        ctx.set_knob("ntt_single_pass", 1)
        x = torch.from_numpy(a.view(np.int64).copy()).to("cuda")
        ctx.ntt([x], 0, len(primes), inverse=False)
        ctx.sync()
        assert np.array_equal(x.cpu().numpy().view(np.uint64).reshape(len(primes), pr.n), A)
        ctx.ntt([x], 0, len(primes), inverse=True)
        ctx.sync()
        assert np.array_equal(x.cpu().numpy().view(np.uint64).reshape(len(primes), pr.n), a)
    del rng


def test_tracer_counts_launches_and_bytes(setup10):
    """The tracer only observes: same bits with it on, and per-class counts
    that match the launch structure of a hoisted rotation."""
    pr, o, keys, ctx = setup10
    _, ct = encrypt(o, keys, pr, 31)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    ctx.sync()
    ctx.trace_read()
    assert ctx.trace_read() == {}                                  # tracer off: nothing recorded
    ctx.set_knob("trace", 1)
    try:
        out = ctx.rotate_hoisted_batch([g], [1, 7])
        tab = ctx.trace_read()
    finally:
        ctx.set_knob("trace", 0)
    for u, s in enumerate([1, 7]):
        assert np.array_equal(ctx.export_ct(out[u]), o.rotate(ct, s, keys).data)
    # one ModUp shared by both steps; both key switches in one step-batched launch per stage
    assert tab["modup_conv"][0] == 1 and tab["ks_inner_steps"][0] == 1 and tab["ks_final_steps"][0] == 1
    assert tab["moddown_conv"][0] == 1 and "ks_inner" not in tab
    N, l, K = pr.n, ct.level, len(pr.p)
    beta = -(-(l + 1) // pr.alpha)
    ne = l + 1 + K
    # the extended digits read once (shared by both steps); per step its key (2 polys per digit,
    # each with its Shoup companions) read and u (2 polys) written
    assert tab["ks_inner_steps"][2] == (beta * ne + 2 * (4 * beta * ne + 2 * ne)) * N * 8
    for name, (n, ms, by) in tab.items():
        assert n > 0 and ms > 0 and by > 0, name


def test_import_export_roundtrip(setup10):
    pr, o, keys, ctx = setup10
    _, ct = encrypt(o, keys, pr, 1)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    assert np.array_equal(ctx.export_ct(g), ct.data)


@pytest.mark.parametrize("level", [4, 3, 1])
def test_rescale_parity(setup10, level):
    pr, o, keys, ctx = setup10
    _, ct = encrypt(o, keys, pr, 2)
    while ct.level > level:
        ct = o.rescale(ct)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    want = o.rescale(ct)
    got = ctx.rescale(g)
    assert got.level == want.level and got.scale == want.scale
    assert np.array_equal(ctx.export_ct(got), want.data)
    # in place
    ctx.rescale(g, out=g)
    assert np.array_equal(ctx.export_ct(g), want.data)


@pytest.mark.parametrize("step", [1, 3, 7, 64, 100, -1, 255])
def test_rotate_parity(setup10, step):
    pr, o, keys, ctx = setup10
    _, ct = encrypt(o, keys, pr, 3)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    assert np.array_equal(ctx.export_ct(ctx.rotate(g, step)), o.rotate(ct, step, keys).data)


def test_rotate_lower_level_and_hoisted(setup10):
    pr, o, keys, ctx = setup10
    _, ct = encrypt(o, keys, pr, 4)
    ct = o.rescale(ct)                                   # level 3: ragged last digit
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    steps = [1, 2, 3, 5, 0]
    outs = ctx.rotate_hoisted(g, steps)
    for s, out in zip(steps, outs):
        assert np.array_equal(ctx.export_ct(out), o.rotate(ct, s, keys).data)
        assert np.array_equal(ctx.export_ct(out), ctx.export_ct(ctx.rotate(g, s)))


@pytest.mark.parametrize("rescales", [0, 2])
def test_square_parity(setup10, rescales):
    pr, o, keys, ctx = setup10
    _, ct = encrypt(o, keys, pr, 5)
    for _ in range(rescales):
        ct = o.rescale(ct)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    got = ctx.square(g)
    want = o.square(ct, keys)
    assert got.scale == want.scale
    assert np.array_equal(ctx.export_ct(got), want.data)


def test_add_parity(setup10):
    pr, o, keys, ctx = setup10
    _, a = encrypt(o, keys, pr, 6)
    _, b = encrypt(o, keys, pr, 7)
    ga, gb = ctx.import_ct(a.data, a.level, a.scale), ctx.import_ct(b.data, b.level, b.scale)
    assert np.array_equal(ctx.export_ct(ctx.add(ga, gb)), o.add(a, b).data)


@pytest.mark.parametrize("m,n,n1,bias", DENSE_CASES)
def test_dense_parity(setup10, m, n, n1, bias):
    pr, o, keys, ctx = setup10
    rng = np.random.default_rng(m * 1000 + n * 10 + n1)
    W = rng.normal(0, 0.05, (m, n))
    b = rng.normal(0, 0.05, m) if bias else None
    x, ct = encrypt(o, keys, pr, 8, width=n)
    lay = o.prepare_dense(W, b, n1, ct.level, ct.scale)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    got = ctx.eval_dense(g, d)
    want = o.dense(ct, lay, keys)
    assert got.scale == want.scale and got.level == want.level
    assert np.array_equal(ctx.export_ct(got), want.data)


@pytest.mark.parametrize("m,n,n1,bias", DENSE_CASES)
def test_dense_qp_parity(setup10, m, n, n1, bias):
    """Lazy-ModDown form (HE_DENSE_QP): diagonals over Q_l u P, inner sums over
    Q_l u P, one ModDown per inner sum, against the oracle's orc_dense_qp."""
    pr, o, keys, ctx = setup10
    rng = np.random.default_rng(m * 1000 + n * 10 + n1 + 1)
    W = rng.normal(0, 0.05, (m, n))
    b = rng.normal(0, 0.05, m) if bias else None
    x, ct = encrypt(o, keys, pr, 9, width=n)
    lay = o.prepare_dense(W, b, n1, ct.level, ct.scale, qp=True)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale, qp=True)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    got = ctx.eval_dense(g, d)
    want = o.dense(ct, lay, keys)
    assert got.scale == want.scale and got.level == want.level
    assert np.array_equal(ctx.export_ct(got), want.data)


@pytest.mark.parametrize("fuse", [1, 0])
def test_dense_qp_lower_level_batched(setup10, fuse):
    """Lazy-ModDown form one level down (the last digit holds one limb),
    three ciphertexts batched: each equals its single call and the oracle;
    with the baby steps' inner product fused into the inner sums (knob
    ks_fuse = 1, the default) and as two launches (0)."""
    pr, o, keys, ctx = setup10
    ctx.set_knob("ks_fuse", fuse)
    m, n, n1 = 8, 64, 8
    W = np.random.default_rng(29).normal(0, 0.05, (m, n))
    b = np.random.default_rng(30).normal(0, 0.05, m)
    cts = [o.rescale(encrypt(o, keys, pr, 50 + i, width=n)[1]) for i in range(3)]
    lay = o.prepare_dense(W, b, n1, cts[0].level, cts[0].scale, qp=True)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale, qp=True)
    gs = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
    batch = ctx.eval_dense_batch(gs, d)
    for i, c in enumerate(cts):
        got = ctx.export_ct(batch[i])
        assert np.array_equal(got, ctx.export_ct(ctx.eval_dense(gs[i], d)))
        assert np.array_equal(got, o.dense(c, lay, keys).data)
    ctx.set_knob("ks_fuse", 1)


@pytest.mark.parametrize("qp", [False, True])
def test_dense_64_baby_steps(qp):
    """The widest baby-step count the workspace takes (n1 = 64: 63 rotations
    in one step-batched key switch), both forms, two ciphertexts batched."""
    pr = small(10)
    m = n = n1 = 64
    o, keys, ctx = make_setup(pr, plan.rotation_steps(m, n, n1), max_batch=2, max_n1=n1, max_n2=1, relin=False)
    W = np.random.default_rng(31).normal(0, 0.05, (m, n))
    b = np.random.default_rng(32).normal(0, 0.05, m)
    cts = [encrypt(o, keys, pr, 60 + i, width=n)[1] for i in range(2)]
    lay = o.prepare_dense(W, b, n1, cts[0].level, cts[0].scale, qp=qp)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale, qp=qp)
    out = ctx.eval_dense_batch([ctx.import_ct(c.data, c.level, c.scale) for c in cts], d)
    for i, c in enumerate(cts):
        assert np.array_equal(ctx.export_ct(out[i]), o.dense(c, lay, keys).data), i


RS_CASES = [(4, 64, 2, False, 2), (4, 64, 2, True, 4), (2, 128, 2, False, 3), (8, 256, 4, True, 3),
            (4, 64, 2, False, 1), (8, 256, 4, True, 1)]


@pytest.fixture(scope="module")
def setup_rs():
    pr = small(10)
    steps = set()
    for m, n, n1, _, rs in RS_CASES:
        steps |= set(plan.rotation_steps(m, n, n1, rs)) | set(plan.rotation_steps(m, n, n1))
    return (pr,) + make_setup(pr, sorted(steps), max_batch=3)


@pytest.mark.parametrize("m,n,n1,qp,rs_bits", RS_CASES)
def test_dense_rotate_sum_hoisted_parity(setup_rs, m, n, n1, qp, rs_bits):
    """Hoisted rotate-and-sum (HE_DENSE_RS): groups of rs_bits bits, each one
    ModUp, the group's rotations fused into one extended sum, one ModDown;
    three ciphertexts batched, against the oracle; rs_bits = 1 also equals
    the sequential form bit for bit."""
    pr, o, keys, ctx = setup_rs
    rng = np.random.default_rng(m + n + n1 + rs_bits)
    W, b = rng.normal(0, 0.05, (m, n)), rng.normal(0, 0.05, m)
    cts = [encrypt(o, keys, pr, 70 + i, width=n)[1] for i in range(3)]
    lay = o.prepare_dense(W, b, n1, cts[0].level, cts[0].scale, qp=qp, rs_bits=rs_bits)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale, qp=qp, rs_bits=rs_bits)
    gs = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
    out = ctx.eval_dense_batch(gs, d)
    for i, c in enumerate(cts):
        got = ctx.export_ct(out[i])
        assert np.array_equal(got, o.dense(c, lay, keys).data), i
    if rs_bits == 1:
        d0 = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale, qp=qp)
        assert np.array_equal(ctx.export_ct(ctx.eval_dense(gs[0], d0)), ctx.export_ct(out[0]))


def test_batched_equals_single(setup10):
    pr, o, keys, ctx = setup10
    m, n, n1 = 8, 64, 4
    W = np.random.default_rng(9).normal(0, 0.05, (m, n))
    b = np.random.default_rng(10).normal(0, 0.05, m)
    cts = [encrypt(o, keys, pr, 20 + i, width=n)[1] for i in range(3)]
    lay = o.prepare_dense(W, b, n1, cts[0].level, cts[0].scale)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale)
    gs = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
    batch = ctx.eval_dense_batch(gs, d)
    sq = ctx.square_batch(batch)
    rs = ctx.rescale_batch(sq)
    for i, c in enumerate(cts):
        single = ctx.rescale(ctx.square(ctx.eval_dense(gs[i], d)))
        assert np.array_equal(ctx.export_ct(rs[i]), ctx.export_ct(single))
        want = o.rescale(o.square(o.dense(c, lay, keys), keys))
        assert np.array_equal(ctx.export_ct(rs[i]), want.data)
    rot = ctx.rotate_hoisted_batch(gs, [1, 7])
    for i, c in enumerate(cts):
        for u, s in enumerate([1, 7]):
            assert np.array_equal(ctx.export_ct(rot[i * 2 + u]), o.rotate(c, s, keys).data)


def test_hoisted_rotation_groups(setup10):
    """More (item, step) pairs than one step-batched switch holds (the
    workspace holds 7 steps; 3 items x 9 steps run as groups of 7 and 2),
    with an identity step (N/2) in the list: every output against the oracle."""
    pr, o, keys, ctx = setup10
    steps = [1, 2, 3, 5, 7, 64, pr.n // 2, 100, -1, 255]
    cts = [encrypt(o, keys, pr, 40 + i)[1] for i in range(3)]
    gs = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
    rot = ctx.rotate_hoisted_batch(gs, steps)
    for i, c in enumerate(cts):
        for u, s in enumerate(steps):
            want = c.data if s == pr.n // 2 else o.rotate(c, s, keys).data
            assert np.array_equal(ctx.export_ct(rot[i * len(steps) + u]), want), (i, s)


def test_full_batch_of_64():
    """The largest batch (64 ciphertexts) through a dense layer, square and
    rescale: every item equals its single-ciphertext evaluation; two items
    against the oracle."""
    pr = small(10)
    m, n, n1 = 8, 64, 4
    o, keys, ctx = make_setup(pr, plan.rotation_steps(m, n, n1), max_batch=64, max_n1=n1, max_n2=m // n1)
    W = np.random.default_rng(19).normal(0, 0.05, (m, n))
    b = np.random.default_rng(20).normal(0, 0.05, m)
    cts = [encrypt(o, keys, pr, 300 + i, width=n)[1] for i in range(64)]
    lay = o.prepare_dense(W, b, n1, cts[0].level, cts[0].scale)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale)
    gs = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
    out = ctx.rescale_batch(ctx.square_batch(ctx.eval_dense_batch(gs, d)))
    for i in range(64):
        single = ctx.rescale(ctx.square(ctx.eval_dense(gs[i], d)))
        assert np.array_equal(ctx.export_ct(out[i]), ctx.export_ct(single)), i
    for i in (0, 63):
        want = o.rescale(o.square(o.dense(cts[i], lay, keys), keys))
        assert np.array_equal(ctx.export_ct(out[i]), want.data)
    # lazy-ModDown form: n2 B = 128 extended inner sums brought down in one set of launches
    lq = o.prepare_dense(W, b, n1, cts[0].level, cts[0].scale, qp=True)
    dq = ctx.dense_load(lq.level, m, n, n1, lq.pts, lq.bias, lq.pt_scale, lq.bias_scale, qp=True)
    outq = ctx.eval_dense_batch(gs, dq)
    for i in (0, 17, 63):
        assert np.array_equal(ctx.export_ct(outq[i]), o.dense(cts[i], lq, keys).data), i


def test_error_codes(setup10):
    he = _he()
    pr, o, keys, ctx = setup10
    _, ct = encrypt(o, keys, pr, 11)
    g = ctx.import_ct(ct.data, ct.level, ct.scale)
    with pytest.raises(he.HeError) as e:
        ctx.rotate(g, 13)                               # no key for step 13
    assert e.value.code == -3
    low = ctx.new_ct(0)
    g0 = ctx.import_ct(np.zeros((2, 1, pr.n), np.uint64), 0, 1.0)
    with pytest.raises(he.HeError) as e:
        ctx.rescale(g0, out=low)
    assert e.value.code == -4
    with pytest.raises(he.HeError) as e:
        he.Context(10, [97], [193], 1)                  # not 1 mod 2N
    assert e.value.code == -2
    with pytest.raises(he.HeError) as e:
        ctx.rotate(g, 1, out=g)                         # output aliases the input
    assert e.value.code == -1
    with pytest.raises(he.HeError) as e:
        ctx.rotate_hoisted_batch([g] * 5, [1])          # more items than the bound batch (4)
    assert e.value.code == -6
    lay_n1 = 16                                         # baby steps beyond the bound workspace (8)
    d = ctx.dense_load(pr.L, 16, 16, lay_n1, np.zeros((16, pr.L + 1, pr.n), np.uint64), None, 1.0, 1.0)
    with pytest.raises(he.HeError) as e:
        ctx.eval_dense(g, d)
    assert e.value.code == -6


def test_network_cfg1_end_to_end():
    """Config 1 at full size: bit-exact ciphertexts and logits within 2^-12 of FP64."""
    pr = params.preset("cfg1")
    steps = ckks.network_steps(pr.layers)
    o, keys, ctx = make_setup(pr, steps, max_batch=2, max_n1=8, max_n2=8)
    Ws, bs = synth.network_weights(pr.layers, pr.sigma_w)
    lays = o.prepare_network(Ws, bs, [l[2] for l in pr.layers])
    dls = [ctx.dense_load(l.level, l.m, l.n, l.n1, l.pts, l.bias, l.pt_scale, l.bias_scale) for l in lays]
    for r in range(2):
        x, ct = encrypt(o, keys, pr, r, width=pr.layers[0][1])
        g = ctx.import_ct(ct.data, ct.level, ct.scale)
        for li, d in enumerate(dls):
            g = ctx.rescale(ctx.eval_dense(g, d))
            if li + 1 < len(dls):
                g = ctx.rescale(ctx.square(g))
        want = o.eval_network(ct, lays, keys)
        got = ctx.export_ct(g)
        assert g.level == want.level and g.scale == want.scale
        assert np.array_equal(got, want.data)
        y = o.decrypt_decode(ckks.Ciphertext(got, g.level, g.scale), keys.sk).real[:2]
        yr = plainnet.forward(x, Ws, bs)
        assert np.max(np.abs(y - yr)) <= 2.0 ** -12
        assert plainnet.predict(y) == plainnet.predict(yr) or abs(yr[0] - yr[1]) < 2.0 ** -11


def test_library_graph_replays():
    """A whole cfg1 network for 3 requests captured by the library
    (he_graph_begin / he_graph_end) and replayed three times, with eager work
    on the same context and new inputs between the replays: every replay
    equals the oracle bit for bit, and the eager work is undisturbed."""
    import torch
    from paper_2104_09164_amd.batch import NetworkRunner
    from paper_2104_09164_amd import netplan
    pr = params.preset("cfg1")
    steps = ckks.network_steps(pr.layers)
    o, keys, ctx = make_setup(pr, steps, max_batch=3, max_n1=8, max_n2=8)
    Ws, bs = synth.network_weights(pr.layers, pr.sigma_w)
    lays = o.prepare_network(Ws, bs, [l[2] for l in pr.layers])
    npl = netplan.plan_network(pr.log_n, pr.q, pr.p, pr.alpha, pr.scale_bits, pr.layers)
    dls = [ctx.dense_load(l.level, l.m, l.n, l.n1, l.pts, l.bias, l.pt_scale, l.bias_scale) for l in lays]
    runner = NetworkRunner(ctx, npl, dls, 3)
    g = runner.capture(3)
    for rep in range(3):
        cts = [encrypt(o, keys, pr, 10 * rep + i, width=pr.layers[0][1])[1] for i in range(3)]
        for i, ct in enumerate(cts):
            runner.inputs[i].buf.copy_(ctx.import_ct(ct.data, ct.level, ct.scale).buf)
        g.replay()
        torch.cuda.synchronize()
        # eager work on the same context between replays
        e = ctx.rescale(ctx.import_ct(cts[0].data, cts[0].level, cts[0].scale))
        assert np.array_equal(ctx.export_ct(e), o.rescale(cts[0]).data)
        for i, ct in enumerate(cts):
            want = o.eval_network(ct, lays, keys)
            out = runner.outputs(3)[i]
            assert out.level == want.level and out.scale == want.scale
            assert np.array_equal(ctx.export_ct(out), want.data), (rep, i)

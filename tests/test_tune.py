"""Autotuner selection logic (CPU); the GPU test checks that knobs never change a bit."""
import json

import numpy as np
import pytest

from paper_2104_09164_amd import tune


def test_n1_candidates():
    assert tune.n1_candidates(128) == [1, 2, 4, 8, 16, 32, 64]
    assert tune.n1_candidates(2) == [1, 2]
    assert tune.n1_candidates(256, 32) == [1, 2, 4, 8, 16, 32]
    for m in (2, 64, 256):
        for n1 in tune.n1_candidates(m):
            assert m % n1 == 0


def test_pick_min_and_batch():
    assert tune.pick_min({"a": 3.0, "b": 1.0, "c": 1.0}) == "b"
    rates = {1: 100.0, 8: 700.0, 16: 1100.0, 32: 1150.0}
    lat = {1: 10.0, 8: 11.4, 16: 14.5, 32: 27.8}
    assert tune.pick_batch(rates, lat, None) == 32
    assert tune.pick_batch(rates, lat, 20.0) == 16
    assert tune.pick_batch(rates, lat, 5.0) == 1


def test_knob_grid_covers_space():
    grid = tune.knob_grid({"a": [1, 2], "b": [3, 4, 5]})
    assert len(grid) == 6 and {json.dumps(g, sort_keys=True) for g in grid} == \
        {json.dumps({"a": a, "b": b}, sort_keys=True) for a in (1, 2) for b in (3, 4, 5)}


@pytest.mark.gpu
def test_knobs_preserve_bits():
    from oracle import ckks, params, plan
    from paper_2104_09164_amd import he, synth
    pr = params.make(14, [50, 40, 40, 40], [50, 50], 2, 30)
    o = ckks.Oracle(pr)
    m, n, n1 = 8, 64, 4
    keys = o.keygen(1, plan.rotation_steps(m, n, n1))
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(3, n1, m // n1)
    ctx.load_keys(keys.rlk, keys.rot)
    W, b = synth.network_weights([(m, n, n1)], 0.05)
    cts = [o.encrypt(plan.input_slots(synth.request_input(n, r), pr.slots), keys.pk, r) for r in range(3)]
    lay = o.prepare_dense(W[0], b[0], n1, pr.L, pr.scale)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale)
    want = [o.rescale(o.square(o.dense(c, lay, keys), keys)).data for c in cts]
    for knobs in tune.knob_grid():
        for k, v in knobs.items():
            ctx.set_knob(k, v)
        gs = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
        out = ctx.rescale_batch(ctx.square_batch(ctx.eval_dense_batch(gs, d)))
        for g, w in zip(out, want):
            assert np.array_equal(ctx.export_ct(g), w), knobs


@pytest.mark.gpu
@pytest.mark.parametrize("m,n,n1,rs", [(8, 64, 8, 0), (8, 64, 4, 2), (8, 64, 2, 0), (16, 64, 2, 3)])
def test_fused_knobs_preserve_bits(m, n, n1, rs):
    """The fused lazy-ModDown inner sums (n2 = 1, 2, 4, 8 giant sums) under
    every setting of ks_fuse_g (requests per thread) and ks_fuse_waves (the
    three-waves-per-SIMD build), and in the LDS-shared form (ks_fuse_lds)
    with one or two position blocks per workgroup (ks_fuse_pair), the
    blocks in address order or along the automorphism (ks_fuse_orbit):
    nine requests (partial last groups: one request in the last workgroup of
    four or eight waves, the others idle), each equal to the oracle bit for
    bit."""
    from oracle import ckks, params, plan
    from paper_2104_09164_amd import he, synth
    pr = params.make(12, [60, 45, 45, 45, 45], [60, 60, 60], 3, 40)
    o = ckks.Oracle(pr)
    keys = o.keygen(1, plan.rotation_steps(m, n, n1, rs))
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(9, n1, m // n1)
    ctx.load_keys(keys.rlk, keys.rot)
    W, b = synth.network_weights([(m, n, n1)], 0.05)
    cts = [o.encrypt(plan.input_slots(synth.request_input(n, r), pr.slots), keys.pk, 70 + r) for r in range(9)]
    lay = o.prepare_dense(W[0], b[0], n1, pr.L, pr.scale, qp=True, rs_bits=rs)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale, qp=True, rs_bits=rs)
    want = [o.dense(c, lay, keys).data for c in cts]
    for g, w, lds, pair, orb in [(0, 0, 0, 0, 1), (1, 0, 0, 0, 1), (0, 3, 0, 0, 1), (1, 3, 0, 0, 1), (0, 0, 4, 0, 1),
                                 (0, 0, 8, 0, 1), (0, 0, 16, 0, 1), (0, 0, 8, 0, 0), (0, 0, 16, 0, 0),
                                 (0, 0, 4, 1, 1), (0, 0, 8, 1, 0)]:
        ctx.set_knob("ks_fuse_g", g)
        ctx.set_knob("ks_fuse_waves", w)
        ctx.set_knob("ks_fuse_lds", lds)
        ctx.set_knob("ks_fuse_pair", pair)
        ctx.set_knob("ks_fuse_orbit", orb)
        gs = [ctx.import_ct(c.data, c.level, c.scale) for c in cts]
        out = ctx.eval_dense_batch(gs, d)
        for i, (x, y) in enumerate(zip(out, want)):
            assert np.array_equal(ctx.export_ct(x), y), (g, w, lds, pair, orb, i)
    ctx.set_knob("ks_fuse_pair", 0)
    ctx.set_knob("ks_fuse_orbit", 1)
    # one request alone in a workgroup of four (three idle waves), the register form for it, and
    # the single-request kernel (values-only streams on the 45-bit primes)
    for mb, one in ((1, 1), (2, 0), (2, 1)):
        ctx.set_knob("ks_fuse_lds", 8)
        ctx.set_knob("ks_fuse_min_batch", mb)
        ctx.set_knob("ks_fuse_one", one)
        g1 = ctx.eval_dense_batch([ctx.import_ct(cts[4].data, cts[4].level, cts[4].scale)], d)
        assert np.array_equal(ctx.export_ct(g1[0]), want[4]), (mb, one)



@pytest.mark.gpu
@pytest.mark.parametrize("qbits,alpha", [(48, 1), (50, 2), (51, 3), (36, 1)])
def test_fused_lds_at_prime_bounds(qbits, alpha):
    """The LDS-shared fused inner sums, and the single-request kernel, on
    primes at the bounds of their forms: just below 2^50 (the last primes of the 28-bit column sums), just
    above it (51-bit primes: the lazy integer sums), 48-bit primes with five
    digits (the widest key sum here), and 36-bit primes; five requests, each
    equal to the oracle bit for bit."""
    from oracle import ckks, params, plan
    from paper_2104_09164_amd import he, synth
    m, n, n1 = 8, 64, 4
    pr = params.make(12, [60] + [qbits] * 4, [60] * 3, alpha, qbits - 5)
    o = ckks.Oracle(pr)
    keys = o.keygen(1, plan.rotation_steps(m, n, n1, 0))
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    ctx.bind(5, n1, m // n1)
    ctx.load_keys(keys.rlk, keys.rot)
    W, b = synth.network_weights([(m, n, n1)], 0.05)
    cts = [o.encrypt(plan.input_slots(synth.request_input(n, r), pr.slots), keys.pk, 90 + r) for r in range(5)]
    lay = o.prepare_dense(W[0], b[0], n1, pr.L, pr.scale, qp=True)
    d = ctx.dense_load(lay.level, m, n, n1, lay.pts, lay.bias, lay.pt_scale, lay.bias_scale, qp=True)
    want = [o.dense(c, lay, keys).data for c in cts]
    out = ctx.eval_dense_batch([ctx.import_ct(c.data, c.level, c.scale) for c in cts], d)
    for i, (x, y) in enumerate(zip(out, want)):
        assert np.array_equal(ctx.export_ct(x), y), (qbits, alpha, i)
    # one request: the single-request kernel (column key sums below 2^50)
    for i in (0, 3):
        g1 = ctx.eval_dense_batch([ctx.import_ct(cts[i].data, cts[i].level, cts[i].scale)], d)
        assert np.array_equal(ctx.export_ct(g1[0]), want[i]), (qbits, alpha, "one", i)

def test_knob_space_is_bit_preserving_and_valid():
    # every tuned key is a documented knob and every value one the library accepts
    assert set(tune.KNOB_SPACE) <= {"ntt_chunk_mb", "ntt_cols", "ntt_cols_b", "ntt_single_pass", "ks_fuse",
                                    "ks_fuse_g", "ks_fuse_waves", "ks_fuse_lds", "ks_fuse_min_batch",
                                    "ks_fuse_pair", "ks_fuse_orbit", "ks_fuse_one"}
    assert set(tune.KNOB_SPACE["ntt_cols"]) <= {8, 16, 32}
    assert set(tune.KNOB_SPACE["ntt_cols_b"]) <= {0, 8, 16, 32}
    assert all(v >= 0 for v in tune.KNOB_SPACE["ntt_chunk_mb"])


@pytest.mark.gpu
def test_knob_api_validation():
    from paper_2104_09164_amd import he
    q, p = he.prime_chain(12, [50, 40], [50])
    ctx = he.Context(12, q, p, 1)
    defaults = {"ntt_chunk_mb": 0, "ntt_cols": 16, "ntt_cols_b": 0, "ntt_single_pass": 0, "ks_fuse": 1,
                "ks_fuse_g": 0, "ks_fuse_waves": 0, "ks_fuse_lds": 8, "ks_fuse_min_batch": 3, "ks_fuse_pair": 0,
                "ks_fuse_orbit": 1, "ks_fuse_one": 1,
                "trace": 0}
    for k, v in defaults.items():
        assert ctx.get_knob(k) == v
    for k, bad in [("ntt_cols", 12), ("ntt_cols_b", 4), ("ntt_single_pass", 2), ("ks_fuse", 2), ("trace", 3),
                   ("ks_fuse_g", 2), ("ks_fuse_waves", 2), ("ks_fuse_lds", 2), ("ks_fuse_min_batch", 0),
                   ("ks_fuse_pair", 2), ("ks_fuse_orbit", 2), ("ks_fuse_one", 2),
                   ("ntt_chunk_mb", -1),
                   ("no_such_knob", 1)]:
        with pytest.raises(he.HeError) as e:
            ctx.set_knob(k, bad)
        assert e.value.code == -1
        if k in defaults:
            assert ctx.get_knob(k) == defaults[k]          # a rejected value leaves the knob unchanged
    ctx.set_knob("ntt_cols_b", 32)
    assert ctx.get_knob("ntt_cols_b") == 32
    # the tracer records nothing while off and everything while on
    assert ctx.trace_read() == {}
    import torch
    x = torch.zeros(2 * (1 << 12), dtype=torch.int64, device="cuda")
    ctx.set_knob("trace", 1)
    ctx.ntt([x], 0, 2, inverse=False)
    tab = ctx.trace_read()
    ctx.set_knob("trace", 0)
    assert tab["ntt_fwd_onepass"][0] == 1 and tab["ntt_fwd_onepass"][2] == 2 * (1 << 12) * 16
    ctx.ntt([x], 0, 2, inverse=False)
    assert ctx.trace_read() == {}

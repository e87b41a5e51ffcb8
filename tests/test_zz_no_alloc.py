"""The rescale that allocates nothing (he_rescale_batch_noalloc), through the
C ABI, against the existing entry point he_rescale_batch and the oracle, bit
for bit: two calls in a row on the same GPU (the static scratch keeps the first
call's contents), the second with fewer ciphertexts at a lower level and in
place; the size limit and the no-workspace case."""
import ctypes as C

import numpy as np
import pytest

from oracle import ckks, params

pytestmark = pytest.mark.gpu


def _cts(ctx, pr, level, count, seed):
    from paper_2104_09164_amd import synth
    N = pr.n
    host = [synth.uniform_residues(pr.q[: level + 1], N, (2,), seed + i) for i in range(count)]
    return host, [ctx.import_ct(h, level, 2.0 ** 40) for h in host]


def test_noalloc_rescale_matches_rescale_batch():
    from paper_2104_09164_amd import he
    pr = params.make(15, [60] + [40] * 6, [60, 60], 2, 40)
    o = ckks.Oracle(pr)
    ctx = he.Context(pr.log_n, pr.q, pr.p, pr.alpha)
    lib = he.lib()
    # first call: 6 ciphertexts at the top level, out of place, no workspace bound yet
    host, cts = _cts(ctx, pr, pr.L, 6, 100)
    outs = [ctx.new_ct(pr.L - 1) for _ in cts]
    ia, oa = ctx._arr(cts), ctx._arr(outs)
    assert lib.he_rescale_batch_noalloc(ctx.h, len(cts), ia, oa) == 0
    ctx._sync_meta(outs, oa)
    ctx.bind(8, 1, 1)
    ref = ctx.rescale_batch(cts)
    for i, (a, b) in enumerate(zip(outs, ref)):
        assert (a.level, a.scale) == (b.level, b.scale)
        ga = ctx.export_ct(a)
        assert np.array_equal(ga, ctx.export_ct(b)), f"item {i}"
        want = o.rescale(ckks.Ciphertext(host[i], pr.L, 2.0 ** 40))
        assert np.array_equal(ga, want.data) and a.scale == want.scale
    # second call right after: 2 ciphertexts one level lower, in place
    host2, cts2 = _cts(ctx, pr, pr.L - 1, 2, 200)
    _, twin = _cts(ctx, pr, pr.L - 1, 2, 200)
    ref2 = ctx.rescale_batch(twin)
    ia2 = ctx._arr(cts2)
    assert lib.he_rescale_batch_noalloc(ctx.h, len(cts2), ia2, ia2) == 0
    ctx._sync_meta(cts2, ia2)
    for i, (a, b) in enumerate(zip(cts2, ref2)):
        assert (a.level, a.scale) == (b.level, b.scale) == (pr.L - 2, 2.0 ** 40 / pr.q[pr.L - 1])
        assert np.array_equal(ctx.export_ct(a), ctx.export_ct(b)), f"in-place item {i}"
    # beyond the static array: refused, nothing enqueued
    many_in, many = _cts(ctx, pr, pr.L, 12, 300)
    outs_m = [ctx.new_ct(pr.L - 1) for _ in many]
    assert lib.he_rescale_batch_noalloc(ctx.h, len(many), ctx._arr(many), ctx._arr(outs_m)) == -6   # HE_ENOMEM
    # level 0 cannot be rescaled
    _, z = _cts(ctx, pr, 0, 1, 400)
    zo = [ctx.new_ct(0)]
    assert lib.he_rescale_batch_noalloc(ctx.h, 1, ctx._arr(z), ctx._arr(zo)) == -4           # HE_ELEVEL
